"""GPU-vs-oracle comparison with the tie protocol.

The oracle records, per seed, the decisions that FP32 arithmetic could take
the other way - a chi2 near the cut, a near rank tie at the k/(k+1) beam
boundary or at the final choice, a propagation near tangency - and keeps
only those whose reversal changes the seed's result (it re-runs the seed
with the decision inverted).  A seed is tie-sensitive when such a relevant
decision lies within eps of its threshold.  Every other seed must have the
identical hit list, and then states, all 15 elements of the local 5x5
covariance and chi2 must agree within the frozen tolerances.  A
tie-sensitive seed whose hits differ must equal the oracle's own outcome of
one of its near decisions taken the other way.
"""
import json
import math
import os

import numpy as np

import oracle
from paper_1702_06359_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
with open(os.path.join(HERE, "tolerances.json")) as _f:
    TOL = json.load(_f)


def local_frame(phi_pos, disk=False):
    """Columns: u along the layer at azimuth phi_pos, then z (cylinder) or r
    (disk, whose plane fixes z), q/pT, phi, theta."""
    G = np.zeros((6, 5))
    G[0, 0], G[1, 0] = -math.sin(phi_pos), math.cos(phi_pos)
    if disk:
        G[0, 1], G[1, 1] = math.cos(phi_pos), math.sin(phi_pos)
    else:
        G[2, 1] = 1.0
    G[3, 2] = G[4, 3] = G[5, 4] = 1.0
    return G


def state_errors(par_g, cov_g, par_o, cov_o, disk=False):
    """Per track, max |dp|/sigma on the 5-D local frame, and max over all 15
    elements of the local 5x5 covariance of |dC_ij| / sqrt(C_ii C_jj) (the
    relative difference on the diagonal), the oracle as reference."""
    n = par_o.shape[0]
    dpar = np.zeros(n)
    dcov = np.zeros(n)
    Cg = synth.unpack_sym(cov_g)
    Co = synth.unpack_sym(cov_o)
    for i in range(n):
        G = local_frame(math.atan2(par_o[i, 1], par_o[i, 0]), disk)
        d = par_g[i] - par_o[i]
        d[4] = (d[4] + np.pi) % (2 * np.pi) - np.pi
        lo = G.T @ Co[i] @ G
        lg = G.T @ Cg[i] @ G
        so = np.diag(lo)
        dpar[i] = np.max(np.abs(G.T @ d) / np.sqrt(so))
        dcov[i] = np.max(np.abs(lg - lo) / np.sqrt(np.outer(so, so)))
    return dpar, dcov


def tie_sensitive(orc, tol):
    return (orc["m_cut"] < tol["eps_cut"]) | (orc["m_rank"] < tol["eps_rank"]) | (orc["m_prop"] < tol["eps_prop"])


def explained_by_alternative(orc_row, hits, status, tol, nl):
    """True when (hits, status) is the oracle's outcome of one of the seed's
    near decisions (within eps) taken the other way."""
    for a in range(int(orc_row["n_alt"])):
        eps = tol["eps_cut"] if orc_row["alt_kind"][a] == 0 else tol["eps_rank"]
        if orc_row["alt_margin"][a] >= eps:
            continue
        if (orc_row["alt_hits"][a][:nl] == hits).all() and orc_row["alt_status"][a] == status:
            return True
    return False


def compare_build(gpu, orc, cfg, hits, seed_par, seed_cov, rows=None, tol=None):
    """gpu: dict of arrays (rows = all seeds, or the `rows` subset); orc:
    oracle structured array for the same rows, in the same order."""
    tol = tol or TOL["build"]
    rows = np.arange(orc.shape[0]) if rows is None else np.asarray(rows)
    nl = cfg.n_layers
    g_hits = gpu["hits"][rows]
    o_hits = orc["hits"][:, :nl]
    same = (g_hits == o_hits).all(axis=1)
    tie = tie_sensitive(orc, tol)
    bad = np.flatnonzero(~same & ~tie)
    rep = dict(n=len(rows), identical=int(same.sum()), tie=int(tie.sum()), tie_differs=int((~same & tie).sum()),
               mismatch=bad.tolist()[:20], n_mismatch=int(len(bad)))
    # counts and status on identical seeds
    s = same
    rep["status_mismatch"] = int((gpu["status"][rows][s] != orc["status"][s]).sum())
    rep["nhits_mismatch"] = int((gpu["n_hits"][rows][s] != orc["n_hits"][s]).sum())
    rep["nholes_mismatch"] = int((gpu["n_holes"][rows][s] != orc["n_holes"][s]).sum())
    dpar, dcov = state_errors(gpu["par"][rows][s], gpu["cov"][rows][s], orc["par"][s], orc["cov"][s],
                              disk=bool(cfg.kind[0]))
    dchi = np.abs(gpu["chi2"][rows][s] - orc["chi2"][s]) / (1.0 + orc["chi2"][s])
    rep["max_dpar_sigma"] = float(dpar.max()) if dpar.size else 0.0
    rep["max_dcov_rel"] = float(dcov.max()) if dcov.size else 0.0
    rep["max_dchi2_rel"] = float(dchi.max()) if dchi.size else 0.0
    rep["p9999_dpar_sigma"] = float(np.quantile(dpar, 0.9999)) if dpar.size else 0.0
    rep["p9999_dcov_rel"] = float(np.quantile(dcov, 0.9999)) if dcov.size else 0.0
    # a tie-sensitive seed that differs must be the oracle's outcome of one of
    # its near decisions taken the other way; otherwise it is reported with
    # its hit list replayed through the oracle
    unexplained = []
    hs = None
    for j in np.flatnonzero(~same & tie):
        i = rows[j]
        if explained_by_alternative(orc[j], gpu["hits"][i], gpu["status"][i], tol, nl):
            continue
        hs = hs or oracle.HitSet(hits)
        lh = gpu["hits"][i]
        tot, per, ok = oracle.replay(cfg, hs, seed_par[i], seed_cov[i], lh)
        unexplained.append(dict(seed=int(i), replay_ok=bool(ok), gpu_status=int(gpu["status"][i]),
                                n_alt=int(orc[j]["n_alt"])))
    rep["tie_invalid"] = unexplained
    return rep


def assert_build_parity(rep, tol=None, max_tie_frac=None):
    tol = tol or TOL["build"]
    max_tie_frac = tol["max_tie_differs_frac"] if max_tie_frac is None else max_tie_frac
    assert rep["n_mismatch"] == 0, rep
    assert rep["status_mismatch"] == 0 and rep["nhits_mismatch"] == 0 and rep["nholes_mismatch"] == 0, rep
    assert rep["max_dpar_sigma"] <= tol["tau_par_sigma"], rep
    assert rep["max_dcov_rel"] <= tol["tau_cov_rel"], rep
    assert rep["max_dchi2_rel"] <= tol["eps_chi2_rel"], rep
    assert not rep["tie_invalid"], rep
    assert rep["tie_differs"] <= max(1, max_tie_frac * rep["n"]), rep
