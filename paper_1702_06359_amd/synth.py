"""Seeded synthetic events for the barrel KF track builder.

This is the *input generator* shared by the tests, the benchmark and the
FP64 oracle's callers.  It holds none of the track builder's arithmetic (no
Kalman propagation, Jacobian, transport, update or chi2): it only simulates
particles and detector hits, and derives the seeds from the first three hits
by plain circle geometry.

The event model is the paper's toy detector (Section 2.2, "Test Scenarios"):
an ideal barrel of concentric cylinders in a uniform longitudinal field,
Gaussian-smeared hit positions and a particle gun with flat transverse
momentum between 0.5 and 10 GeV, no correlations between particles.  The
workload additions (material of 0.2 % X0 per layer, uniform noise hits,
pseudo-rapidity range, vertex spread, 3-hit truth seeds) are the synthetic
stand-ins for the paper's simulated events.

Units: cm, GeV, tesla, radians.  Field along +z.  A track state is
(x, y, z, q/pT, phi, theta) with phi the azimuth of the momentum and theta
its polar angle.

Random streams: numpy PCG64 seeded by SeedSequence([1702, 6359, cfg, event]);
independent child streams are spawned for kinematics, vertex, multiple
scattering, hit smearing, noise and the per-layer hit shuffle.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

KAPPA = 0.00299792458  # GeV / (T cm): transverse momentum = KAPPA * B * radius

# seed covariance, in the local frame (u along the layer, z, q/pT, phi, theta);
# chosen a little wider than the measured spread of the 3-hit circle estimate
# (u and z: the third hit itself; q/pT: sagitta over an 8 cm chord, sigma_rphi
# = 100 um; phi and theta: chord directions), so the seed is conservative.
SEED_SIGMA = (0.012, 0.12, 0.20, 0.009, 0.020)
# the same for disks, frame (u along r*phi, v along r, q/pT, phi, theta): the
# three seed hits span only a few cm of transverse path, so the curvature is
# nearly unknown (measured spreads on generated endcap events: 0.010, 0.10,
# 0.48, 0.011, 0.0066)
SEED_SIGMA_DISK = (0.012, 0.12, 0.58, 0.014, 0.008)
# and their correlations, measured on the same events: the short arc ties the
# curvature to the direction
SEED_CORR_DISK = np.array([
    [1.00, 0.00, -0.34, 0.55, 0.00],
    [0.00, 1.00, 0.00, 0.00, 0.70],
    [-0.34, 0.00, 1.00, -0.93, 0.00],
    [0.55, 0.00, -0.93, 1.00, 0.00],
    [0.00, 0.70, 0.00, 0.00, 1.00],
])
# loose prior for a fit that starts from the innermost hit (second
# coordinate: z on a cylinder, r on a disk)
PRIOR_SIGMA = (1.0, 10.0, 1.0, 0.1, 0.1)


@dataclasses.dataclass
class Geometry:
    """Ideal barrel: n_layers cylinders at radius r_L, each 0.2 % X0 thick.

    With disk_z set the layers are instead endcap disks (Section 2.2: the
    CMS geometry's endcaps, here ideal planes): disk L lies in the plane
    z = disk_z[L] between radii disk_rmin and radii[L]; its hits are measured
    along r*phi (sigma_rphi) and r (sigma_r)."""
    n_layers: int = 10
    radii: Sequence[float] = tuple(4.0 * (i + 1) for i in range(10))
    x0: Sequence[float] = tuple(0.002 for _ in range(10))
    bz: float = 3.8
    sigma_rphi: float = 0.01
    sigma_z: float = 0.1
    mass: float = 0.13957
    disk_z: Optional[Sequence[float]] = None
    disk_rmin: float = 2.0
    sigma_r: float = 0.1
    # finite thickness (Section 2.2's simplified geometry: modules of a layer
    # sit at different radii, or z on a disk): a track's hit on layer L lies
    # on the surface r_L + d (z_L + d), d uniform in [-t/2, t/2] per crossing
    thickness: Optional[Sequence[float]] = None

    @property
    def is_disk(self) -> bool:
        return self.disk_z is not None

    def thick(self, L: int) -> float:
        return 0.0 if self.thickness is None else float(self.thickness[L])

    @staticmethod
    def endcap(n_layers: int = 10) -> "Geometry":
        """Forward tracker of n_layers disks at z = 30, 40, ... cm, radii 2-60 cm."""
        return Geometry(n_layers=n_layers, radii=tuple(60.0 for _ in range(n_layers)),
                        x0=tuple(0.002 for _ in range(n_layers)),
                        disk_z=tuple(30.0 + 10.0 * i for i in range(n_layers)))

    def half_z(self) -> np.ndarray:
        """Half length that bounds noise hits and the bin grid (|eta| < 1 plus
        margin); for disks, the outer radius."""
        r = np.asarray(self.radii, dtype=np.float64)
        if self.is_disk:
            return r.copy()
        return 1.05 * r * math.sinh(1.0) + 3.0


@dataclasses.dataclass
class Event:
    geometry: Geometry
    hits: List[np.ndarray]             # per layer (n_L, 3) float64 x, y, z (caller order)
    seed_par: np.ndarray               # (n_s, 6) float64, state at the third seed layer
    seed_cov: np.ndarray               # (n_s, 21) float64 packed upper triangle
    seed_hits: np.ndarray              # (n_s, 3) int32 hit index per seed layer
    truth_hit: np.ndarray              # (n_t, n_layers) int32 index of the track's hit, -1 if none
    truth_par: np.ndarray              # (n_t, n_layers, 6) true state at each crossing (before the kick)
    vertex_par: np.ndarray             # (n_t, 6) true state at the vertex
    prior_par: np.ndarray              # (n_t, 6) loose prior at the innermost hit (for a fit)
    prior_cov: np.ndarray              # (n_t, 21)
    n_noise: np.ndarray                # (n_layers,) noise hits per layer

    @property
    def n_seeds(self) -> int:
        return int(self.seed_par.shape[0])

    @property
    def n_hits_total(self) -> int:
        return int(sum(h.shape[0] for h in self.hits))


def _streams(cfg: int, event: int, n: int):
    ss = np.random.SeedSequence([1702, 6359, int(cfg), int(event)])
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(n)]


def _cross_cylinder(x, y, z, qpt, phi, theta, r, bz):
    """First forward crossing of the cylinder of radius r by a helix.

    Simulation-side geometry written in the turning-angle form: the position
    after turning by angle a is centre + (sin(phi+a), -cos(phi+a))/w with
    w = -KAPPA*B*q/pT, and the crossing angle solves a single sine equation.
    Returns the new (x, y, z, phi) and the transverse path length.
    """
    w = -KAPPA * bz * qpt
    straight = np.abs(w) < 1e-12
    ws = np.where(straight, 1.0, w)
    cx = x - np.sin(phi) / ws
    cy = y + np.cos(phi) / ws
    cn = np.hypot(cx, cy)
    # |c|^2 + 1/w^2 + (2/w) (cx sin psi - cy cos psi) = r^2
    k = (r * r - cn * cn - 1.0 / (ws * ws)) * ws / 2.0
    ratio = np.clip(k / np.where(cn > 0, cn, 1.0), -1.0, 1.0)
    beta = np.arctan2(-cy, cx)   # cx sin psi - cy cos psi = cn sin(psi + beta)
    two_pi = 2.0 * np.pi
    best = np.full(np.shape(x), np.inf)
    for psi in (np.arcsin(ratio) - beta, np.pi - np.arcsin(ratio) - beta):
        d = psi - phi
        d = np.where(w > 0, np.mod(d, two_pi), -np.mod(-d, two_pi))
        s = d / ws
        s = np.where(s <= 1e-9, s + two_pi / np.abs(ws), s)
        best = np.minimum(best, s)
    s_helix = best
    # straight line: |p + s u|^2 = r^2
    b = x * np.cos(phi) + y * np.sin(phi)
    c = x * x + y * y - r * r
    s_line = -b + np.sqrt(np.maximum(b * b - c, 0.0))
    s = np.where(straight, s_line, s_helix)
    a = np.where(straight, 0.0, w * s)
    nphi = phi + a
    nx = np.where(straight, x + s * np.cos(phi), cx + np.sin(nphi) / ws)
    ny = np.where(straight, y + s * np.sin(phi), cy - np.cos(nphi) / ws)
    nz = z + s / np.tan(theta)
    nphi = np.mod(nphi + np.pi, two_pi) - np.pi
    return nx, ny, nz, nphi, s


def _cross_plane(x, y, z, qpt, phi, theta, zd, bz):
    """Crossing of the plane z = zd by a helix: the transverse path is fixed by
    the dip angle, s = (zd - z) tan(theta), and the turning-angle form gives
    the point.  Returns the new (x, y, z, phi) and s (negative: plane behind)."""
    w = -KAPPA * bz * qpt
    straight = np.abs(w) < 1e-12
    ws = np.where(straight, 1.0, w)
    s = (zd - z) * np.tan(theta)
    nphi = phi + np.where(straight, 0.0, w * s)
    cx = x - np.sin(phi) / ws
    cy = y + np.cos(phi) / ws
    nx = np.where(straight, x + s * np.cos(phi), cx + np.sin(nphi) / ws)
    ny = np.where(straight, y + s * np.sin(phi), cy - np.cos(nphi) / ws)
    nphi = np.mod(nphi + np.pi, 2.0 * np.pi) - np.pi
    return nx, ny, np.broadcast_to(np.asarray(zd, dtype=np.float64), np.shape(x)).copy(), nphi, s


def _highland(p, beta, t):
    return 0.0136 / (beta * p) * np.sqrt(t) * (1.0 + 0.038 * np.log(t))


def _circle_seed(p1, p2, p3, z1, z3, bz, at_first: bool):
    """Helix parameters from three points by plain circle geometry."""
    d12 = p2 - p1
    d23 = p3 - p2
    d13 = p3 - p1
    cross = d12[:, 0] * d13[:, 1] - d12[:, 1] * d13[:, 0]
    l12 = np.hypot(d12[:, 0], d12[:, 1])
    l23 = np.hypot(d23[:, 0], d23[:, 1])
    l13 = np.hypot(d13[:, 0], d13[:, 1])
    w = 2.0 * cross / (l12 * l23 * l13)   # signed curvature, >0 = counter-clockwise
    qpt = -w / (KAPPA * bz)

    def half_turn(chord):
        return np.arcsin(np.clip(w * chord / 2.0, -1.0, 1.0))

    def arc(chord):
        t = w * chord / 2.0
        small = np.abs(t) < 1e-8
        return np.where(small, chord, 2.0 * np.arcsin(np.clip(t, -1, 1)) / np.where(small, 1.0, w))

    if at_first:
        phi = np.arctan2(d12[:, 1], d12[:, 0]) - half_turn(l12)
    else:
        phi = np.arctan2(d23[:, 1], d23[:, 0]) + half_turn(l23)
    cot = (z3 - z1) / arc(l13)
    theta = 0.5 * np.pi - np.arctan(cot)
    phi = np.mod(phi + np.pi, 2 * np.pi) - np.pi
    return qpt, phi, theta


def local_cov_to_packed_disk(phi_pos: np.ndarray, sig: Sequence[float],
                             corr: Optional[np.ndarray] = None) -> np.ndarray:
    """As local_cov_to_packed for a disk: the local covariance
    diag(sig) corr diag(sig) (corr = identity by default) in the frame
    (u along r*phi, v along r, q/pT, phi, theta), rotated to global
    coordinates (x = -sin(phi_pos) u + cos(phi_pos) v, y = cos u + sin v);
    z is fixed by the plane and carries no variance."""
    sg = np.asarray(sig, dtype=np.float64)
    R = np.eye(5) if corr is None else np.asarray(corr, dtype=np.float64)
    local = sg[:, None] * R * sg[None, :]
    s = np.sin(phi_pos)
    c = np.cos(phi_pos)
    G = np.zeros((phi_pos.shape[0], 6, 5))
    G[:, 0, 0], G[:, 1, 0] = -s, c
    G[:, 0, 1], G[:, 1, 1] = c, s
    G[:, 3, 2] = G[:, 4, 3] = G[:, 5, 4] = 1.0
    full = G @ local @ np.swapaxes(G, 1, 2)
    return pack_sym(full)


def local_cov_to_packed(phi_pos: np.ndarray, sig: Sequence[float]) -> np.ndarray:
    """Diagonal covariance in the frame (u, z, q/pT, phi, theta) of the layer
    tangent at azimuth phi_pos, expressed in global (x, y, z, q/pT, phi, theta)
    and packed as the 21-entry upper triangle.  This is a change of frame, not
    a filter step: x = x_h - sin(phi_pos) u, y = y_h + cos(phi_pos) u."""
    n = phi_pos.shape[0]
    su, sz, sq, sp, st = sig
    s = np.sin(phi_pos)
    c = np.cos(phi_pos)
    full = np.zeros((n, 6, 6))
    full[:, 0, 0] = s * s * su * su
    full[:, 0, 1] = full[:, 1, 0] = -s * c * su * su
    full[:, 1, 1] = c * c * su * su
    full[:, 2, 2] = sz * sz
    full[:, 3, 3] = sq * sq
    full[:, 4, 4] = sp * sp
    full[:, 5, 5] = st * st
    return pack_sym(full)


def pack_sym(full: np.ndarray) -> np.ndarray:
    iu = np.triu_indices(6)
    return np.ascontiguousarray(full[..., iu[0], iu[1]])


def unpack_sym(packed: np.ndarray) -> np.ndarray:
    iu = np.triu_indices(6)
    out = np.zeros(packed.shape[:-1] + (6, 6))
    out[..., iu[0], iu[1]] = packed
    out[..., iu[1], iu[0]] = packed
    return out


def make_event(n_tracks: int, *, cfg: int = 0, event: int = 0,
               noise: float | Sequence[float] = 0.0,
               geometry: Optional[Geometry] = None,
               smear: bool = True, scatter: bool = True,
               smear_scale: float = 1.0,
               pt_range=(0.5, 10.0), eta_max: float = 1.0,
               vertex_sigma=(0.01, 1.0), eta_range: Optional[Sequence[float]] = None) -> Event:
    """Generate one event of n_tracks particles plus uniform noise hits.

    noise: fraction of the true-hit count added per layer as uniform noise
    (a scalar, or one value per layer).  Pseudo-rapidity: uniform in
    eta_range, by default (-eta_max, eta_max) for a barrel and (1.6, 2.6) for
    the endcap geometry (every track crosses every disk).
    """
    g = geometry or Geometry()
    nl = g.n_layers
    rk, rv, rms, rsm, rno, rsh, rth = _streams(cfg, event, 7)
    n = int(n_tracks)
    pt = rk.uniform(pt_range[0], pt_range[1], n)
    if eta_range is None:
        eta_range = (1.6, 2.6) if g.is_disk else (-eta_max, eta_max)
    eta = rk.uniform(eta_range[0], eta_range[1], n)
    phi = rk.uniform(-np.pi, np.pi, n)
    q = np.where(rk.uniform(0.0, 1.0, n) < 0.5, -1.0, 1.0)
    theta = 2.0 * np.arctan(np.exp(-eta))
    x = rv.normal(0.0, vertex_sigma[0], n)
    y = rv.normal(0.0, vertex_sigma[0], n)
    z = rv.normal(0.0, vertex_sigma[1], n)
    qpt = q / pt
    p = pt / np.sin(theta)
    vertex = np.stack([x, y, z, qpt, phi, theta], axis=1)

    truth = np.zeros((n, nl, 6))
    true_xyz = np.zeros((n, nl, 3))
    for L in range(nl):
        r = float(g.radii[L])
        t = g.thick(L)
        d = rth.uniform(-0.5 * t, 0.5 * t, n) if t > 0 else 0.0
        if g.is_disk:
            x, y, z, phi, _ = _cross_plane(x, y, z, qpt, phi, theta, float(g.disk_z[L]) + d, g.bz)
        else:
            r = r + d
            x, y, z, phi, _ = _cross_cylinder(x, y, z, qpt, phi, theta, r, g.bz)
        truth[:, L] = np.stack([x, y, z, qpt, phi, theta], axis=1)
        phi_pos = np.arctan2(y, x)
        if g.is_disk:
            # r*phi and r measured on the plane
            r_pos = np.hypot(x, y)
            if smear:
                phi_h = phi_pos + rsm.normal(0.0, g.sigma_rphi * smear_scale, n) / r_pos
                r_h = r_pos + rsm.normal(0.0, g.sigma_r * smear_scale, n)
            else:
                phi_h, r_h = phi_pos, r_pos
            true_xyz[:, L] = np.stack([r_h * np.cos(phi_h), r_h * np.sin(phi_h), z], axis=1)
        else:
            if smear:
                phi_h = phi_pos + rsm.normal(0.0, g.sigma_rphi * smear_scale, n) / r
                z_h = z + rsm.normal(0.0, g.sigma_z * smear_scale, n)
            else:
                phi_h = phi_pos
                z_h = z.copy()
            true_xyz[:, L] = np.stack([r * np.cos(phi_h), r * np.sin(phi_h), z_h], axis=1)
        if scatter and g.x0[L] > 0:
            # two independent Gaussian angles in the planes orthogonal to p;
            # path factor 1/|cos| of the angle to the surface normal
            if g.is_disk:
                cos_a = np.abs(np.cos(theta))
            else:
                cos_a = np.abs(np.sin(theta) * np.cos(phi - phi_pos))
            tx = g.x0[L] / np.maximum(cos_a, 1e-6)
            beta = p / np.sqrt(p * p + g.mass * g.mass)
            th0 = _highland(p, beta, tx)
            a1 = rms.normal(0.0, 1.0, n) * th0
            a2 = rms.normal(0.0, 1.0, n) * th0
            d = np.stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)], 1)
            e1 = np.stack([-np.sin(phi), np.cos(phi), np.zeros(n)], 1)
            e2 = np.stack([np.cos(theta) * np.cos(phi), np.cos(theta) * np.sin(phi), -np.sin(theta)], 1)
            d = d + a1[:, None] * e1 + a2[:, None] * e2
            d /= np.linalg.norm(d, axis=1, keepdims=True)
            phi = np.arctan2(d[:, 1], d[:, 0])
            theta = np.arccos(np.clip(d[:, 2], -1.0, 1.0))
            qpt = q / (p * np.sin(theta))

    # noise and per-layer shuffle
    frac = np.broadcast_to(np.asarray(noise, dtype=np.float64), (nl,))
    hz = g.half_z()
    hits = []
    truth_hit = np.zeros((n, nl), dtype=np.int32)
    n_noise = np.zeros(nl, dtype=np.int64)
    for L in range(nl):
        r = float(g.radii[L])
        nn = int(round(frac[L] * n))
        n_noise[L] = nn
        ph = rno.uniform(-np.pi, np.pi, nn)
        t = g.thick(L)
        if g.is_disk:   # uniform over the annulus
            rr = np.sqrt(rno.uniform(g.disk_rmin ** 2, r * r, nn))
            zd = float(g.disk_z[L]) + (rno.uniform(-0.5 * t, 0.5 * t, nn) if t > 0 else 0.0)
            noise_xyz = np.stack([rr * np.cos(ph), rr * np.sin(ph), np.broadcast_to(zd, (nn,))], axis=1)
        else:
            zz = rno.uniform(-hz[L], hz[L], nn)
            rr = r + (rno.uniform(-0.5 * t, 0.5 * t, nn) if t > 0 else 0.0)
            noise_xyz = np.stack([rr * np.cos(ph), rr * np.sin(ph), zz], axis=1)
        allh = np.concatenate([true_xyz[:, L], noise_xyz], axis=0)
        perm = rsh.permutation(allh.shape[0])
        inv = np.empty_like(perm)
        inv[perm] = np.arange(perm.shape[0])
        hits.append(np.ascontiguousarray(allh[perm]))
        truth_hit[:, L] = inv[:n].astype(np.int32)

    # seeds: circle through the first three hits, state at the third hit
    h0, h1, h2 = true_xyz[:, 0], true_xyz[:, 1], true_xyz[:, 2]
    sq, sphi, sth = _circle_seed(h0[:, :2], h1[:, :2], h2[:, :2], h0[:, 2], h2[:, 2], g.bz, False)
    seed_par = np.stack([h2[:, 0], h2[:, 1], h2[:, 2], sq, sphi, sth], axis=1)
    to_packed = local_cov_to_packed_disk if g.is_disk else local_cov_to_packed
    if g.is_disk:
        seed_cov = local_cov_to_packed_disk(np.arctan2(h2[:, 1], h2[:, 0]), SEED_SIGMA_DISK, SEED_CORR_DISK)
    else:
        seed_cov = local_cov_to_packed(np.arctan2(h2[:, 1], h2[:, 0]), SEED_SIGMA)
    seed_hits = np.ascontiguousarray(truth_hit[:, :3])
    pq, pphi, pth = _circle_seed(h0[:, :2], h1[:, :2], h2[:, :2], h0[:, 2], h2[:, 2], g.bz, True)
    prior_par = np.stack([h0[:, 0], h0[:, 1], h0[:, 2], pq, pphi, pth], axis=1)
    prior_cov = to_packed(np.arctan2(h0[:, 1], h0[:, 0]), PRIOR_SIGMA)
    return Event(geometry=g, hits=hits, seed_par=np.ascontiguousarray(seed_par),
                 seed_cov=seed_cov, seed_hits=seed_hits, truth_hit=truth_hit,
                 truth_par=truth, vertex_par=vertex, prior_par=np.ascontiguousarray(prior_par),
                 prior_cov=prior_cov, n_noise=n_noise)


# ---- workload recipes --------------------------------------------------------

def best_hit_event(n_tracks: int = 1000, event: int = 0) -> Event:
    """1,000 tracks, no noise: the best-hit (one candidate per seed) workload."""
    return make_event(n_tracks, cfg=0, event=event, noise=0.0)


def ckf_events(n_events: int = 10, n_tracks: int = 20000, noise: float = 0.10, first: int = 0):
    """Events of the combinatorial workload: 20,000 tracks, 10 % noise hits per layer."""
    return [make_event(n_tracks, cfg=1, event=first + e, noise=noise) for e in range(n_events)]


def endcap_events(n_events: int = 10, n_tracks: int = 10000, noise: float = 0.10, first: int = 0):
    """Events of the endcap workload: ten disks, 1.6 < eta < 2.6, 10 % noise
    hits per disk.  10,000 tracks per event carry the particle density per
    unit of eta of the 20,000-track barrel workload (|eta| < 1)."""
    g = Geometry.endcap()
    return [make_event(n_tracks, cfg=3, event=first + e, noise=noise, geometry=g) for e in range(n_events)]


def fit_batch_sizes(n_batches: int = 64, total: int = 1_000_000, lo: int = 2000, hi: int = 30000,
                    seed: int = 0) -> np.ndarray:
    """Uneven batch sizes in [lo, hi] summing exactly to total."""
    rng = _streams(2, 10_000 + seed, 1)[0]
    u = rng.integers(lo, hi + 1, n_batches)
    while u.sum() != total:
        i = int(rng.integers(0, n_batches))
        if u.sum() > total and u[i] > lo:
            u[i] -= 1
        elif u.sum() < total and u[i] < hi:
            u[i] += 1
    return u.astype(np.int64)


def loguniform_sizes(n: int, lo: int, hi: int, cfg: int, seed: int = 0) -> np.ndarray:
    rng = _streams(cfg, 20_000 + seed, 1)[0]
    return np.round(np.exp(rng.uniform(math.log(lo), math.log(hi), n))).astype(np.int64)


def batched_events(n_events: int = 256, lo: int = 500, hi: int = 20000, first: int = 0):
    """Uneven events: track counts log-uniform in [lo, hi], noise U[0.1, 0.5] per (event, layer)."""
    sizes = loguniform_sizes(n_events, lo, hi, cfg=3, seed=first)
    rng = _streams(3, 30_000 + first, 1)[0]
    out = []
    for e in range(n_events):
        f = rng.uniform(0.1, 0.5, 10)
        out.append(make_event(int(sizes[e]), cfg=3, event=first + e, noise=f))
    return out


def event_truth_tracks(ev: Event) -> np.ndarray:
    return ev.truth_hit
