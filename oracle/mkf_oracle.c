/* FP64 CPU oracle of the Kalman-filter track builder and fitter (barrel
 * cylinders and endcap disks).
 *
 * TEST INFRASTRUCTURE ONLY: the tests, the package smoke check and the
 * benchmark's CPU-baseline leg call it; the GPU library never does, and the
 * two share no code.  Plain scalar double, generic small-matrix loops, brute
 * force over every hit of a layer, no blocking or fusion: written to be read
 * against the method, not to be fast.
 *
 * What it follows (Cerati et al., "Kalman filter tracking on parallel
 * architectures"):
 *  - Section 2: three stages; building projects each candidate outward layer
 *    by layer, collects compatible hits with the KF and branches to several
 *    candidates per seed; fitting repeats the KF over a fixed hit set.
 *  - Section 2.2: ideal barrel, uniform longitudinal field, hybrid state
 *    (global Cartesian position, polar momentum), KF update on the plane
 *    tangent to the hit radius; the simplified geometry's endcap disks are
 *    planes at fixed z, reached by propagation to that z.
 *  - Section 3.2.1: a variable number of hit candidates per layer, so the
 *    beam is re-ranked and pruned after every layer.
 * Where the paper gives no formula, the readings used are: helix in a uniform
 * field with signed q/pT; Highland multiple scattering added when leaving a
 * layer; 2-D (r*phi, z) measurement; strict chi2 < cut; hole child only when
 * no hit was accepted; beam order (n_hits desc, chi2 asc, parent rank asc,
 * hit index asc, hole last); hits must lie in the forward half-space of the
 * predicted point.
 */
#include "mkf_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdatomic.h>
#include <stdlib.h>
#include <string.h>

#define KAPPA 0.00299792458   /* GeV / (T cm) */
#define HOLE_ID 0x7fffffff

static const double PI = 3.14159265358979323846;

/* ---------------------------------------------------------------- helpers */

static double wrap_angle(double a)
{
    while (a > PI) a -= 2.0 * PI;
    while (a <= -PI) a += 2.0 * PI;
    return a;
}

static void unpack21(const double *p, double C[36])
{
    int k = 0;
    for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) {
            C[i * 6 + j] = p[k];
            C[j * 6 + i] = p[k];
            ++k;
        }
}

static void pack21(const double C[36], double *p)
{
    int k = 0;
    for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) p[k++] = C[i * 6 + j];
}

/* generic dense product: out[m x n] = A[m x k] B[k x n] */
static void matmul(const double *A, const double *B, double *out, int m, int k, int n)
{
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int t = 0; t < k; ++t) acc += A[i * k + t] * B[t * n + j];
            out[i * n + j] = acc;
        }
}

static void transpose(const double *A, double *out, int m, int n)
{
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) out[j * m + i] = A[i * n + j];
}

static void symmetrize(double C[36])
{
    for (int i = 0; i < 6; ++i)
        for (int j = i + 1; j < 6; ++j) {
            double v = 0.5 * (C[i * 6 + j] + C[j * 6 + i]);
            C[i * 6 + j] = v;
            C[j * 6 + i] = v;
        }
}

/* ------------------------------------------------------------ propagation */

/* Helix in a uniform field B along z.  With w = -KAPPA*B*q/pT the momentum
 * azimuth turns as phi(s) = phi + w*s over transverse path s, so
 *   x(s) = x + s*A(a),  y(s) = y + s*B(a),  a = w*s,
 *   A = (sin(phi+a) - sin phi)/a,  B = (cos phi - cos(phi+a))/a,
 * and z(s) = z + s*cot(theta).  The small-|a| limits are taken by series. */
static void sinc_terms(double a, double *S1, double *C1, double *S2, double *C2)
{
    if (fabs(a) < 1e-2) {
        double a2 = a * a;
        *S1 = 1.0 - a2 / 6.0 + a2 * a2 / 120.0;                   /* sin a / a        */
        *C1 = a / 2.0 - a * a2 / 24.0 + a * a2 * a2 / 720.0;       /* (1 - cos a) / a  */
        *S2 = -a / 3.0 + a * a2 / 30.0 - a * a2 * a2 / 840.0;      /* (a cos a - sin a)/a^2 */
        *C2 = 0.5 - a2 / 8.0 + a2 * a2 / 144.0;                    /* (a sin a - 1 + cos a)/a^2 */
    } else {
        double sa = sin(a), ca = cos(a);
        *S1 = sa / a;
        *C1 = (1.0 - ca) / a;
        *S2 = (a * ca - sa) / (a * a);
        *C2 = (a * sa - 1.0 + ca) / (a * a);
    }
}

/* State after transverse path s along the helix, and (F != NULL) its
 * derivative with respect to the input state once the path is tied to the
 * surface: kind 0 the cylinder of radius r (x^2 + y^2 = r^2 at the end),
 * kind 1 the plane z = const. */
static int helix_to(const double p[6], double s, double bz, int kind, double r, double out[6],
                    double F[36], double *path)
{
    const double x = p[0], y = p[1], z = p[2], qpt = p[3], phi = p[4], th = p[5];
    const double w = -KAPPA * bz * qpt;
    double a = w * s, S1, C1, S2, C2;
    sinc_terms(a, &S1, &C1, &S2, &C2);
    const double cph = cos(phi), sph = sin(phi);
    const double A = cph * S1 - sph * C1;        /* (sin(phi+a) - sin phi)/a */
    const double B = cph * C1 + sph * S1;        /* (cos phi - cos(phi+a))/a */
    const double gx = cph * S2 - sph * C2;       /* d A / d a */
    const double gy = sph * S2 + cph * C2;       /* d B / d a */
    const double cot = cos(th) / sin(th);
    const double nx = x + s * A, ny = y + s * B;
    const double nphi = phi + a;
    (void)r;

    out[0] = nx;
    out[1] = ny;
    out[2] = z + s * cot;
    out[3] = qpt;
    out[4] = wrap_angle(nphi);
    out[5] = th;
    if (path) *path = s;
    if (!F) return 0;

    /* d(out)/d(in) at fixed path s */
    double P[36];
    memset(P, 0, sizeof(P));
    for (int i = 0; i < 6; ++i) P[i * 6 + i] = 1.0;
    const double dw = -KAPPA * bz;                /* dw / d(q/pT) */
    P[0 * 6 + 3] = s * s * gx * dw;
    P[0 * 6 + 4] = -s * B;
    P[1 * 6 + 3] = s * s * gy * dw;
    P[1 * 6 + 4] = s * A;
    P[2 * 6 + 5] = -s / (sin(th) * sin(th));
    P[4 * 6 + 3] = s * dw;
    /* the path itself depends on the inputs through the surface equation;
     * t is d(out)/ds */
    const double cn = cos(nphi), sn = sin(nphi);
    const double t[6] = {cn, sn, cot, 0.0, w, 0.0};
    double ds[6];
    if (kind == 0) {           /* x(s)^2 + y(s)^2 = r^2 */
        const double den = nx * cn + ny * sn;
        for (int j = 0; j < 6; ++j) ds[j] = -(nx * P[0 * 6 + j] + ny * P[1 * 6 + j]) / den;
    } else {                   /* z(s) = const */
        for (int j = 0; j < 6; ++j) ds[j] = -P[2 * 6 + j] / cot;
    }
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) F[i * 6 + j] = P[i * 6 + j] + t[i] * ds[j];
    return 0;
}

/* Intersections of the track's transverse circle with the circle |P| = r.
 * The track circle passes through p0 = (x, y) with tangent t = (cos phi,
 * sin phi); its centre is c = p0 + n / w with n = (-sin phi, cos phi) the left
 * normal, its radius 1/|w|.  Two circles meet on their radical line, the
 * points with equal power |P|^2 - r^2 = |P - c|^2 - 1/w^2; the 1/w^2 terms
 * cancel exactly, and multiplied by w the line reads
 *   P . m = q,   m = w p0 + n,   q = w (|p0|^2 + r^2) / 2 + p0 . n,
 * which for w = 0 is the track's own straight line (the line-circle case).
 * The line meets |P| = r at the foot point (q / |m|^2) m plus or minus the
 * half chord h along m's perpendicular, h^2 = r^2 - q^2 / |m|^2.  Returns the
 * number of points (0 or 2) and the signed margin r - |q| / |m| (zero at
 * tangency, negative when the circles do not meet). */
static int circle_points(const double p[6], double r, double w, double P[2][2], double *margin)
{
    const double x = p[0], y = p[1], cph = cos(p[4]), sph = sin(p[4]);
    const double nx = -sph, ny = cph;
    const double mx = w * x + nx, my = w * y + ny;
    const double m2 = mx * mx + my * my;
    const double q = 0.5 * w * (x * x + y * y + r * r) + (x * nx + y * ny);
    if (!(m2 > 0.0)) {          /* concentric circles: no crossing point */
        *margin = 0.0;
        return 0;
    }
    const double mn = sqrt(m2);
    const double dist = q / mn;
    *margin = r - fabs(dist);
    const double h2 = r * r - dist * dist;
    if (h2 < 0.0) return 0;
    const double h = sqrt(h2);
    const double fx = dist * mx / mn, fy = dist * my / mn;    /* foot point */
    const double ux = -my / mn, uy = mx / mn;                 /* along the line */
    P[0][0] = fx + h * ux;
    P[0][1] = fy + h * uy;
    P[1][0] = fx - h * ux;
    P[1][1] = fy - h * uy;
    return 2;
}

/* Signed transverse path from p0 to a point P of the track circle, with the
 * turning angle in (-pi, pi]: the displacement d = P - p0 has components
 * d.t = sin(a) / w and d.n = (1 - cos a) / w for a turn a = w s, so
 * a = atan2(w d.t, 1 - w d.n); at w = 0 the path is d.t. */
static double path_to_point(const double p[6], double w, const double P[2], double *turn)
{
    const double cph = cos(p[4]), sph = sin(p[4]);
    const double dx = P[0] - p[0], dy = P[1] - p[1];
    const double dt = dx * cph + dy * sph, dn = -dx * sph + dy * cph;
    if (w == 0.0) {
        *turn = 0.0;
        return dt;
    }
    const double a = atan2(w * dt, 1.0 - w * dn);
    *turn = a;
    return a / w;
}

int orc_propagate(const double p[6], double r, double bz, double out[6], double F[36],
                  double *path, double *margin)
{
    const double w = -KAPPA * bz * p[3];
    double P[2][2], mrg;
    const int np = circle_points(p, r, w, P, &mrg);
    if (margin) *margin = mrg;
    /* the first crossing ahead: every point is reached after a positive path,
     * a turn of up to one full revolution in the sense of w */
    double s = -1.0;
    int best = -1;
    for (int i = 0; i < np; ++i) {
        double a, si = path_to_point(p, w, P[i], &a);
        if (w > 0.0 && a <= 0.0) si = (a + 2.0 * PI) / w;
        else if (w < 0.0 && a >= 0.0) si = (a - 2.0 * PI) / w;
        if (si > 1e-12 * r && (best < 0 || si < s)) {
            s = si;
            best = i;
        }
    }
    if (best < 0) return 1;
    helix_to(p, s, bz, 0, r, out, F, path);
    out[0] = P[best][0];         /* the crossing point itself, on the cylinder */
    out[1] = P[best][1];
    return 0;
}

/* Propagation to the plane z = zd (an endcap disk of the simplified
 * geometry, Section 2.2): the longitudinal
 * motion is linear in the transverse path, z(s) = z + s cot(theta), so
 * s = (zd - z) tan(theta), valid when positive (the helix moves towards the
 * plane).  *margin receives s. */
int orc_propagate_plane(const double p[6], double zd, double bz, double out[6], double F[36],
                        double *path, double *margin)
{
    const double s = (zd - p[2]) * tan(p[5]);
    if (margin) *margin = s;
    if (!(s > 0.0) || !isfinite(s)) return 1;
    helix_to(p, s, bz, 1, 0.0, out, F, path);
    out[2] = zd;                 /* on the plane by definition, not up to rounding */
    return 0;
}

/* Second step of the two-step propagation (Section 2.2: from the layer's
 * average radius or z to the exact surface of a hit): the crossing of the
 * cylinder of radius `where` (kind 0) or of the plane z = `where` (kind 1)
 * nearest along the helix, ahead of the state or behind it.  On a cylinder,
 * of the two crossing points of the circles, each reached by a turn of at
 * most half a revolution either way, the one of smaller |s|.  Returns 1 when
 * the helix never reaches the surface. */
int orc_step_near(const double p[6], int kind, double where, double bz, double out[6], double F[36],
                  double *path)
{
    double s;
    if (kind == 1) {
        s = (where - p[2]) * tan(p[5]);
        if (!isfinite(s)) return 1;
        helix_to(p, s, bz, 1, 0.0, out, F, path);
        out[2] = where;
        return 0;
    }
    const double w = -KAPPA * bz * p[3];
    double P[2][2], mrg;
    const int np = circle_points(p, where, w, P, &mrg);
    int best = -1;
    s = 0.0;
    for (int i = 0; i < np; ++i) {
        double a;
        const double si = path_to_point(p, w, P[i], &a);    /* principal turn, either sign */
        if (best < 0 || fabs(si) < fabs(s)) {
            s = si;
            best = i;
        }
    }
    if (best < 0) return 1;
    helix_to(p, s, bz, 0, where, out, F, path);
    out[0] = P[best][0];
    out[1] = P[best][1];
    return 0;
}

void orc_transport(const double F[36], double C[36])
{
    double FC[36], Ft[36];
    matmul(F, C, FC, 6, 6, 6);
    transpose(F, Ft, 6, 6);
    matmul(FC, Ft, C, 6, 6, 6);
    symmetrize(C);
}

/* ------------------------------------------------------------ material */

/* Highland scattering angle for a layer of x0 radiation lengths crossed at
 * incidence alpha to its normal (the radial direction on a cylinder, z on a
 * disk); the two projected angles add noise to the momentum direction:
 * Var phi += th0^2/sin^2 theta, Var theta += th0^2, and q/pT = q/(p sin theta)
 * picks up the theta part at fixed |p|. */
void orc_add_ms(const double p[6], int kind, double x0, double mass, double C[36])
{
    if (x0 <= 0.0) return;
    const double qpt = p[3], phi = p[4], th = p[5];
    const double phipos = atan2(p[1], p[0]);
    double cosa = kind == 0 ? fabs(sin(th) * cos(phi - phipos)) : fabs(cos(th));
    if (cosa < 1e-6) cosa = 1e-6;
    const double t = x0 / cosa;
    const double k = fabs(qpt) * sin(th);                 /* 1 / |p| */
    const double inv_beta_p = k * sqrt(1.0 + mass * mass * k * k);
    const double th0 = 0.0136 * inv_beta_p * sqrt(t) * (1.0 + 0.038 * log(t));
    const double v = th0 * th0;
    const double cot = cos(th) / sin(th);
    /* Q = J diag(v, v) J^T with J the derivative of (q/pT, phi, theta) wrt
     * the two projected angles at fixed |p| */
    double J[12];          /* rows: state params 0..5, cols: (angle_1, angle_2) */
    memset(J, 0, sizeof(J));
    J[4 * 2 + 0] = 1.0 / sin(th);
    J[5 * 2 + 1] = 1.0;
    J[3 * 2 + 1] = -qpt * cot;
    double Jt[12], JJt[36];
    transpose(J, Jt, 6, 2);
    matmul(J, Jt, JJt, 6, 2, 6);
    for (int i = 0; i < 36; ++i) C[i] += v * JJt[i];
}

/* ------------------------------------------------------------ measurement */

/* The measurement is the hit position in a plane through the hit: on a
 * cylinder (kind 0) the tangent plane, coordinates u along
 * (-sin phi_h, cos phi_h, 0) and z; on a disk (kind 1) the disk's own plane,
 * coordinates u and v along (cos phi_h, sin phi_h, 0), the radial direction.
 * H is the 2x6 matrix of that projection, V = diag(sigma_rphi^2, s2^2) with
 * s2 the resolution of the second coordinate. */
static void measurement(const double p[6], const double hit[3], int kind, double srphi, double s2,
                        double H[12], double res[2], double V[4])
{
    const double phih = atan2(hit[1], hit[0]);
    const double sh = sin(phih), ch = cos(phih);
    memset(H, 0, 12 * sizeof(double));
    H[0 * 6 + 0] = -sh;
    H[0 * 6 + 1] = ch;
    res[0] = (hit[0] - p[0]) * (-sh) + (hit[1] - p[1]) * ch;
    if (kind == 0) {
        H[1 * 6 + 2] = 1.0;
        res[1] = hit[2] - p[2];
    } else {
        H[1 * 6 + 0] = ch;
        H[1 * 6 + 1] = sh;
        res[1] = (hit[0] - p[0]) * ch + (hit[1] - p[1]) * sh;
    }
    V[0] = srphi * srphi;
    V[1] = 0.0;
    V[2] = 0.0;
    V[3] = s2 * s2;
}

static void innovation(const double C[36], const double H[12], const double V[4], double HC[12],
                       double S[4], double Sinv[4])
{
    double Ht[12];
    matmul(H, C, HC, 2, 6, 6);
    transpose(H, Ht, 2, 6);
    matmul(HC, Ht, S, 2, 6, 2);
    for (int i = 0; i < 4; ++i) S[i] += V[i];
    const double det = S[0] * S[3] - S[1] * S[2];
    Sinv[0] = S[3] / det;
    Sinv[1] = -S[1] / det;
    Sinv[2] = -S[2] / det;
    Sinv[3] = S[0] / det;
}

double orc_chi2(const double p[6], const double C[36], const double hit[3], int kind, double srphi,
                double s2)
{
    double H[12], r[2], V[4], HC[12], S[4], Si[4], Sr[2];
    measurement(p, hit, kind, srphi, s2, H, r, V);
    innovation(C, H, V, HC, S, Si);
    matmul(Si, r, Sr, 2, 2, 1);
    return r[0] * Sr[0] + r[1] * Sr[1];
}

double orc_update(const double p[6], const double C[36], const double hit[3], int kind, double srphi,
                  double s2, double out_p[6], double out_C[36])
{
    double H[12], r[2], V[4], HC[12], S[4], Si[4], Sr[2];
    measurement(p, hit, kind, srphi, s2, H, r, V);
    innovation(C, H, V, HC, S, Si);
    matmul(Si, r, Sr, 2, 2, 1);
    const double chi2 = r[0] * Sr[0] + r[1] * Sr[1];
    /* gain K = C H^T S^-1 = (H C)^T S^-1 */
    double CHt[12], K[12], Kr[6], KHC[36];
    transpose(HC, CHt, 2, 6);
    matmul(CHt, Si, K, 6, 2, 2);
    matmul(K, r, Kr, 6, 2, 1);
    matmul(K, HC, KHC, 6, 2, 6);
    double np[6], nC[36];
    for (int i = 0; i < 6; ++i) np[i] = p[i] + Kr[i];
    np[4] = wrap_angle(np[4]);
    for (int i = 0; i < 36; ++i) nC[i] = C[i] - KHC[i];
    symmetrize(nC);
    memcpy(out_p, np, sizeof(np));
    memcpy(out_C, nC, sizeof(nC));
    return chi2;
}

/* ------------------------------------------------------------ layers */

/* Propagation to layer L: its cylinder, or its disk's plane. */
static int to_layer(const orc_config *cfg, int L, const double p[6], double out[6], double F[36],
                    double *margin)
{
    if (cfg->kind[L] == 0) return orc_propagate(p, cfg->radius[L], cfg->bz, out, F, NULL, margin);
    return orc_propagate_plane(p, cfg->zplane[L], cfg->bz, out, F, NULL, margin);
}

/* resolution of a layer's second measured coordinate: z or r */
static double second_sigma(const orc_config *cfg, int L)
{
    return cfg->kind[L] == 0 ? cfg->sigma_z : cfg->sigma_r;
}

static double layer_chi2(const orc_config *cfg, int L, const double p[6], const double C[36],
                         const double hit[3])
{
    if (cfg->update3d) return orc_chi2_3d(p, C, hit, cfg->sigma_rphi, cfg->sigma_r, cfg->sigma_z);
    return orc_chi2(p, C, hit, cfg->kind[L], cfg->sigma_rphi, second_sigma(cfg, L));
}

static double layer_update(const orc_config *cfg, int L, const double p[6], const double C[36],
                           const double hit[3], double out_p[6], double out_C[36])
{
    if (cfg->update3d) return orc_update_3d(p, C, hit, cfg->sigma_rphi, cfg->sigma_r, cfg->sigma_z, out_p, out_C);
    return orc_update(p, C, hit, cfg->kind[L], cfg->sigma_rphi, second_sigma(cfg, L), out_p, out_C);
}

static void leave_layer(const orc_config *cfg, int L, const double p[6], double C[36])
{
    orc_add_ms(p, cfg->kind[L], cfg->x0[L], cfg->mass, C);
}

/* The surface of a hit on layer L: its radius on a cylinder, its z on a disk. */
static double hit_surface(const orc_config *cfg, int L, const double hit[3])
{
    return cfg->kind[L] == 0 ? hypot(hit[0], hit[1]) : hit[2];
}

/* Second step on a layer of finite thickness: the state (p, C) on the
 * layer's average surface carried to the hit's own surface.  Returns 1 when
 * the helix does not reach it. */
static int step_to_hit(const orc_config *cfg, int L, const double p[6], const double C[36],
                       const double hit[3], double out_p[6], double out_C[36])
{
    double F[36], np[6], nC[36];
    if (orc_step_near(p, cfg->kind[L], hit_surface(cfg, L, hit), cfg->bz, np, F, NULL)) return 1;
    memcpy(nC, C, sizeof(nC));
    orc_transport(F, nC);
    memcpy(out_p, np, sizeof(np));
    memcpy(out_C, nC, sizeof(nC));
    return 0;
}

/* Fit: straight to the surface of the layer's hit (h != NULL) on a thick
 * layer - the composition of the two steps - else to the average surface. */
static int fit_to_layer(const orc_config *cfg, int L, const double p[6], const double *hit, double out[6],
                        double F[36])
{
    if (hit && cfg->thick[L] > 0.0) {
        if (cfg->kind[L] == 0) return orc_propagate(p, hypot(hit[0], hit[1]), cfg->bz, out, F, NULL, NULL);
        return orc_propagate_plane(p, hit[2], cfg->bz, out, F, NULL, NULL);
    }
    return to_layer(cfg, L, p, out, F, NULL);
}

/* The 3x3 global-Cartesian variant: the measurement is the hit's position
 * (x, y, z) itself, H = [I3 0], with the hit's error ellipsoid
 * V = sigma_rphi^2 u u^T + sigma_r^2 n n^T + sigma_z^2 e_z e_z^T, where
 * u = (-sin phi_h, cos phi_h, 0) and n = (cos phi_h, sin phi_h, 0).  With
 * sigma_r (cylinders) or sigma_z (disks) along the layer normal, it needs
 * all three positive. */
static void measurement3(const double p[6], const double hit[3], double su, double sr, double sz, double H[18],
                         double res[3], double V[9])
{
    const double phih = atan2(hit[1], hit[0]);
    const double u[3] = {-sin(phih), cos(phih), 0.0}, n[3] = {cos(phih), sin(phih), 0.0}, e[3] = {0.0, 0.0, 1.0};
    memset(H, 0, 18 * sizeof(double));
    for (int i = 0; i < 3; ++i) {
        H[i * 6 + i] = 1.0;
        res[i] = hit[i] - p[i];
        for (int j = 0; j < 3; ++j) V[i * 3 + j] = su * su * u[i] * u[j] + sr * sr * n[i] * n[j] + sz * sz * e[i] * e[j];
    }
}

/* inverse of a 3x3 matrix by its cofactors */
static void inverse3(const double A[9], double B[9])
{
    B[0] = A[4] * A[8] - A[5] * A[7];
    B[1] = A[2] * A[7] - A[1] * A[8];
    B[2] = A[1] * A[5] - A[2] * A[4];
    B[3] = A[5] * A[6] - A[3] * A[8];
    B[4] = A[0] * A[8] - A[2] * A[6];
    B[5] = A[2] * A[3] - A[0] * A[5];
    B[6] = A[3] * A[7] - A[4] * A[6];
    B[7] = A[1] * A[6] - A[0] * A[7];
    B[8] = A[0] * A[4] - A[1] * A[3];
    const double det = A[0] * B[0] + A[1] * B[3] + A[2] * B[6];
    for (int i = 0; i < 9; ++i) B[i] /= det;
}

static double update3_impl(const double p[6], const double C[36], const double hit[3], double su, double sr,
                           double sz, double *out_p, double *out_C)
{
    double H[18], r[3], V[9], HC[18], Ht[18], S[9], Si[9], Sr[3];
    measurement3(p, hit, su, sr, sz, H, r, V);
    matmul(H, C, HC, 3, 6, 6);
    transpose(H, Ht, 3, 6);
    matmul(HC, Ht, S, 3, 6, 3);
    for (int i = 0; i < 9; ++i) S[i] += V[i];
    inverse3(S, Si);
    matmul(Si, r, Sr, 3, 3, 1);
    const double chi2 = r[0] * Sr[0] + r[1] * Sr[1] + r[2] * Sr[2];
    if (!out_p) return chi2;
    double CHt[18], K[18], Kr[6], KHC[36], np[6], nC[36];
    transpose(HC, CHt, 3, 6);
    matmul(CHt, Si, K, 6, 3, 3);
    matmul(K, r, Kr, 6, 3, 1);
    matmul(K, HC, KHC, 6, 3, 6);
    for (int i = 0; i < 6; ++i) np[i] = p[i] + Kr[i];
    np[4] = wrap_angle(np[4]);
    for (int i = 0; i < 36; ++i) nC[i] = C[i] - KHC[i];
    symmetrize(nC);
    memcpy(out_p, np, sizeof(np));
    memcpy(out_C, nC, sizeof(nC));
    return chi2;
}

double orc_chi2_3d(const double p[6], const double C[36], const double hit[3], double srphi, double sr, double sz)
{
    return update3_impl(p, C, hit, srphi, sr, sz, NULL, NULL);
}

double orc_update_3d(const double p[6], const double C[36], const double hit[3], double srphi, double sr, double sz,
                     double out_p[6], double out_C[36])
{
    return update3_impl(p, C, hit, srphi, sr, sz, out_p, out_C);
}

/* ------------------------------------------------------------ threading */

typedef struct {
    void (*fn)(void *ctx, int64_t i);
    void *ctx;
    int64_t n;
    int64_t chunk;
    atomic_long next;
} pool_job;

static void *pool_worker(void *arg)
{
    pool_job *job = (pool_job *)arg;
    for (;;) {
        int64_t b = atomic_fetch_add(&job->next, job->chunk);
        if (b >= job->n) break;
        int64_t e = b + job->chunk < job->n ? b + job->chunk : job->n;
        for (int64_t i = b; i < e; ++i) job->fn(job->ctx, i);
    }
    return NULL;
}

static void parallel_for(int64_t n, int n_threads, int64_t chunk, void (*fn)(void *, int64_t), void *ctx)
{
    pool_job job;
    job.fn = fn;
    job.ctx = ctx;
    job.n = n;
    job.chunk = chunk;
    atomic_init(&job.next, 0);
    if (n_threads <= 1) {
        pool_worker(&job);
        return;
    }
    pthread_t th[256];
    if (n_threads > 256) n_threads = 256;
    for (int t = 0; t < n_threads; ++t) pthread_create(&th[t], NULL, pool_worker, &job);
    for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
}

/* ------------------------------------------------------------ fit */

typedef struct {
    const orc_config *cfg;
    const orc_hits *hits;
    const double *init_par, *init_cov;
    const int32_t *track_hits;
    double *out_par, *out_cov, *out_chi2, *hit_chi2;
    int32_t *out_ndof, *out_status;
} fit_ctx;

static void fit_one(void *vctx, int64_t i)
{
    const fit_ctx *c = (const fit_ctx *)vctx;
    const orc_config *cfg = c->cfg;
    const int nl = cfg->n_layers;
    double p[6], C[36], op[6], oC[36];
    memcpy(p, c->init_par + 6 * i, sizeof(p));
    unpack21(c->init_cov + 21 * i, C);
    memcpy(op, p, sizeof(p));
    memcpy(oC, C, sizeof(C));
    double chi2 = 0.0;
    int nupd = 0, status = 0;
    for (int L = 0; L < nl; ++L) {
        if (c->hit_chi2) c->hit_chi2[i * nl + L] = -1.0;
    }
    for (int L = 0; L < nl; ++L) {
        const int32_t h = c->track_hits[i * nl + L];
        const double *hit = h >= 0 ? c->hits->xyz[L] + 3 * (int64_t)h : NULL;
        if (L > 0) {
            double np[6], F[36];
            leave_layer(cfg, L - 1, p, C);
            if (fit_to_layer(cfg, L, p, hit, np, F)) {
                status = 2;
                break;
            }
            memcpy(p, np, sizeof(p));
            orc_transport(F, C);
        }
        if (h >= 0) {
            double c2 = layer_update(cfg, L, p, C, hit, p, C);
            chi2 += c2;
            ++nupd;
            memcpy(op, p, sizeof(p));
            memcpy(oC, C, sizeof(C));
            if (c->hit_chi2) c->hit_chi2[i * nl + L] = c2;
        }
    }
    memcpy(c->out_par + 6 * i, op, sizeof(op));
    pack21(oC, c->out_cov + 21 * i);
    c->out_chi2[i] = chi2;
    c->out_ndof[i] = 2 * nupd - 5;
    c->out_status[i] = status;
}

void orc_fit(const orc_config *cfg, const orc_hits *hits, int32_t n_tracks, const double *init_par,
             const double *init_cov, const int32_t *track_hits, double *out_par, double *out_cov,
             double *out_chi2, int32_t *out_ndof, int32_t *out_status, double *hit_chi2,
             int32_t n_threads)
{
    fit_ctx c = {cfg, hits, init_par, init_cov, track_hits, out_par, out_cov, out_chi2, hit_chi2,
                 out_ndof, out_status};
    parallel_for(n_tracks, n_threads, 64, fit_one, &c);
}

/* ------------------------------------------------------------ fit prior */

void orc_circle_prior(const orc_config *cfg, const orc_hits *hits, int32_t n_tracks,
                      const int32_t *track_hits, const double sig[5], double *out_par, double *out_cov,
                      int32_t *out_ok)
{
    const int nl = cfg->n_layers;
    for (int32_t i = 0; i < n_tracks; ++i) {
        double *par = out_par + 6 * (int64_t)i, *cov = out_cov + 21 * (int64_t)i;
        memset(par, 0, 6 * sizeof(double));
        memset(cov, 0, 21 * sizeof(double));
        out_ok[i] = 0;
        const double *p[3];
        int missing = 0;
        for (int L = 0; L < 3; ++L) {
            const int32_t h = track_hits[(int64_t)i * nl + L];
            if (h < 0) missing = 1;
            else p[L] = hits->xyz[L] + 3 * (int64_t)h;
        }
        if (missing) continue;
        /* transverse circle through the three points: signed curvature from
         * the triangle (twice its signed area over the product of its sides) */
        const double ax = p[1][0] - p[0][0], ay = p[1][1] - p[0][1];
        const double bx = p[2][0] - p[1][0], by = p[2][1] - p[1][1];
        const double cx = p[2][0] - p[0][0], cy = p[2][1] - p[0][1];
        const double area2 = ax * cy - ay * cx;
        const double la = hypot(ax, ay), lb = hypot(bx, by), lc = hypot(cx, cy);
        if (!(la > 0 && lb > 0 && lc > 0) || area2 == 0.0) continue;
        const double w = 2.0 * area2 / (la * lb * lc);        /* > 0: counter-clockwise */
        /* the chord to the second point turns by half the arc's angle from
         * the tangent at the first point */
        const double phi = wrap_angle(atan2(ay, ax) - asin(fmax(-1.0, fmin(1.0, 0.5 * w * la))));
        /* arc length from the first to the third point, z linear in it */
        const double t = 0.5 * w * lc;
        const double arc = fabs(t) < 1e-12 ? lc : 2.0 * asin(fmax(-1.0, fmin(1.0, t))) / w;
        const double cot = (p[2][2] - p[0][2]) / arc;
        par[0] = p[0][0];
        par[1] = p[0][1];
        par[2] = p[0][2];
        par[3] = -w / (KAPPA * cfg->bz);
        par[4] = phi;
        par[5] = 0.5 * PI - atan(cot);
        /* covariance: local diagonal rotated to (x, y) by the hit's azimuth;
         * the second coordinate is z on a cylinder, r on a disk (where the
         * plane fixes z) */
        const double a = atan2(p[0][1], p[0][0]);
        const double s = sin(a), c = cos(a);
        double C[36];
        memset(C, 0, sizeof(C));
        const double vu = sig[0] * sig[0], v2 = sig[1] * sig[1];
        if (cfg->kind[0] == 0) {
            C[0] = s * s * vu;
            C[1] = C[6] = -s * c * vu;
            C[7] = c * c * vu;
            C[14] = v2;
        } else {
            C[0] = s * s * vu + c * c * v2;
            C[1] = C[6] = -s * c * vu + s * c * v2;
            C[7] = c * c * vu + s * s * v2;
        }
        C[21] = sig[2] * sig[2];
        C[28] = sig[3] * sig[3];
        C[35] = sig[4] * sig[4];
        pack21(C, cov);
        out_ok[i] = 1;
    }
}

/* ------------------------------------------------------------ building */

typedef struct {
    double par[6];
    double C[36];
    double chi2;
    int32_t hits[ORC_MAX_LAYERS];
    int32_t n_hits, n_holes, status, stopped;
} cand_t;

enum { KIND_HIT = 0, KIND_HOLE = 1, KIND_STOPPED = 2 };

typedef struct {
    int32_t n_hits;
    double chi2;        /* parent's chi2 plus this hit's chi2 */
    double hit_chi2;
    int32_t parent;     /* parent's rank in the current beam */
    int32_t hit;        /* hit index in the layer, HOLE_ID for holes and stopped */
    int32_t kind;
} entry_t;

static int entry_cmp(const void *va, const void *vb)
{
    const entry_t *a = (const entry_t *)va, *b = (const entry_t *)vb;
    if (a->n_hits != b->n_hits) return a->n_hits > b->n_hits ? -1 : 1;
    if (a->chi2 != b->chi2) return a->chi2 < b->chi2 ? -1 : 1;
    if (a->parent != b->parent) return a->parent < b->parent ? -1 : 1;
    if (a->hit != b->hit) return a->hit < b->hit ? -1 : 1;
    return 0;
}

typedef struct {
    const orc_config *cfg;
    const orc_hits *hits;
    const double *seed_par, *seed_cov;
    const int32_t *seed_hits, *seed_ids;
    orc_track *out;
    orc_track *beam;    /* optional: [n_sel][max_cands], every rank of the final beam */
} build_ctx;

typedef struct {
    cand_t c[ORC_MAX_CANDS];
    int n;
} beam_t;

/* A decision of the beam search that FP32 arithmetic could take the other
 * way: kind 0, the cut on hit `hit` for beam candidate `cand` on `layer`;
 * kind 1, the choice between the k-th and (k+1)-th entries of `layer`;
 * kind 2, the final choice between ranks 0 and 1. */
typedef struct {
    int32_t layer, cand, hit, kind;
    double margin;
} decision_t;

/* What the main run of a seed records: margins, counters, the near
 * decisions and the beam before every layer. */
typedef struct {
    double m_cut_raw, m_cut_far, m_rank_raw, m_rank_far, m_prop;
    int64_t n_prop, n_accept, n_update;
    decision_t *dec;
    int n_dec, cap_dec;
    beam_t *snap;
} run_log;

static void note_decision(run_log *log, int layer, int cand, int hit, int kind, double margin)
{
    if (log->n_dec == log->cap_dec) {
        log->cap_dec = log->cap_dec ? 2 * log->cap_dec : 16;
        log->dec = (decision_t *)realloc(log->dec, log->cap_dec * sizeof(decision_t));
    }
    decision_t *d = &log->dec[log->n_dec++];
    d->layer = layer;
    d->cand = cand;
    d->hit = hit;
    d->kind = kind;
    d->margin = margin;
}

static entry_t *push_entry(entry_t **ent, int *ne, int *cap)
{
    if (*ne == *cap) {
        *cap *= 2;
        *ent = (entry_t *)realloc(*ent, *cap * sizeof(entry_t));
    }
    return &(*ent)[(*ne)++];
}

/* The beam search over layers L0 .. n_layers-1 from beam b (updated in
 * place).  `flip` (may be NULL) takes one decision the other way; `log`
 * (NULL in those re-runs) records margins, counters, near decisions and the
 * beam before each layer. */
static void run_layers(const build_ctx *bc, int L0, beam_t *b, const decision_t *flip, run_log *log)
{
    const orc_config *cfg = bc->cfg;
    const int nl = cfg->n_layers;
    int k = cfg->max_cands;
    if (k > ORC_MAX_CANDS) k = ORC_MAX_CANDS;
    cand_t next[ORC_MAX_CANDS];
    double pred_par[ORC_MAX_CANDS][6], pred_C[ORC_MAX_CANDS][36];
    int cap = 64, ne = 0;
    entry_t *ent = (entry_t *)malloc(cap * sizeof(entry_t));

    for (int L = L0; L < nl; ++L) {
        if (log) log->snap[L] = *b;
        ne = 0;
        const double r = cfg->radius[L];
        for (int c = 0; c < b->n; ++c) {
            cand_t *cd = &b->c[c];
            if (!cd->stopped) {
                double p[6], C[36], F[36], mrg;
                memcpy(p, cd->par, sizeof(p));
                memcpy(C, cd->C, sizeof(C));
                leave_layer(cfg, L - 1, p, C);
                if (log) ++log->n_prop;
                int fail = to_layer(cfg, L, p, pred_par[c], F, &mrg);
                if (log && fabs(mrg) / r < log->m_prop) log->m_prop = fabs(mrg) / r;
                if (fail) {
                    cd->stopped = 1;
                    cd->status = 2;       /* keeps its state on the previous surface */
                } else {
                    memcpy(pred_C[c], C, sizeof(C));
                    orc_transport(F, pred_C[c]);
                    int nacc = 0;
                    const double *xyz = bc->hits->xyz[L];
                    const double *pp = pred_par[c];
                    for (int32_t j = 0; j < bc->hits->n_hits[L]; ++j) {
                        const double *h = xyz + 3 * (int64_t)j;
                        if (h[0] * pp[0] + h[1] * pp[1] <= 0.0) continue;   /* other side */
                        double c2;
                        if (cfg->thick[L] > 0.0) {
                            /* two-step: from the average surface to the hit's */
                            double hp[6], hC[36];
                            if (step_to_hit(cfg, L, pp, pred_C[c], h, hp, hC)) continue;
                            c2 = layer_chi2(cfg, L, hp, hC, h);
                        } else {
                            c2 = layer_chi2(cfg, L, pp, pred_C[c], h);
                        }
                        const double dm = fabs(c2 - cfg->chi2_cut);
                        if (log) {
                            if (dm < log->m_cut_raw) log->m_cut_raw = dm;
                            if (dm < ORC_CUT_CONSIDER) note_decision(log, L, c, j, 0, dm);
                            else if (dm < log->m_cut_far) log->m_cut_far = dm;
                        }
                        int accept = c2 < cfg->chi2_cut;
                        if (flip && flip->kind == 0 && flip->layer == L && flip->cand == c && flip->hit == j)
                            accept = !accept;
                        if (accept) {
                            entry_t *e = push_entry(&ent, &ne, &cap);
                            e->n_hits = cd->n_hits + 1;
                            e->chi2 = cd->chi2 + c2;
                            e->hit_chi2 = c2;
                            e->parent = c;
                            e->hit = j;
                            e->kind = KIND_HIT;
                            ++nacc;
                        }
                    }
                    if (log) log->n_accept += nacc;
                    if (nacc == 0 || cfg->hole_always) {
                        if (cd->n_holes < cfg->max_holes) {
                            entry_t *e = push_entry(&ent, &ne, &cap);
                            e->n_hits = cd->n_hits;
                            e->chi2 = cd->chi2;
                            e->hit_chi2 = 0.0;
                            e->parent = c;
                            e->hit = HOLE_ID;
                            e->kind = KIND_HOLE;
                        } else if (nacc == 0) {
                            /* no hit and no hole left: stop on this surface */
                            cd->stopped = 1;
                            cd->status = 1;
                            memcpy(cd->par, pred_par[c], sizeof(cd->par));
                            memcpy(cd->C, pred_C[c], sizeof(cd->C));
                        }
                    }
                }
            }
            if (cd->stopped) {
                entry_t *e = push_entry(&ent, &ne, &cap);
                e->n_hits = cd->n_hits;
                e->chi2 = cd->chi2;
                e->hit_chi2 = 0.0;
                e->parent = c;
                e->hit = HOLE_ID;
                e->kind = KIND_STOPPED;
            }
        }
        qsort(ent, ne, sizeof(entry_t), entry_cmp);
        if (ne > k && ent[k - 1].n_hits == ent[k].n_hits) {
            const double gap = (ent[k].chi2 - ent[k - 1].chi2) / (1.0 + ent[k - 1].chi2);
            if (log) {
                if (gap < log->m_rank_raw) log->m_rank_raw = gap;
                if (gap < ORC_RANK_CONSIDER) note_decision(log, L, -1, -1, 1, gap);
                else if (gap < log->m_rank_far) log->m_rank_far = gap;
            }
            if (flip && flip->kind == 1 && flip->layer == L) {
                const entry_t t = ent[k - 1];
                ent[k - 1] = ent[k];
                ent[k] = t;
            }
        }
        const int nn = ne < k ? ne : k;
        for (int i = 0; i < nn; ++i) {
            const entry_t *e = &ent[i];
            const cand_t *par = &b->c[e->parent];
            cand_t *nc = &next[i];
            *nc = *par;
            if (e->kind == KIND_HIT) {
                const double *h = bc->hits->xyz[L] + 3 * (int64_t)e->hit;
                if (cfg->thick[L] > 0.0) {
                    double hp[6], hC[36];
                    step_to_hit(cfg, L, pred_par[e->parent], pred_C[e->parent], h, hp, hC);
                    layer_update(cfg, L, hp, hC, h, nc->par, nc->C);
                } else {
                    layer_update(cfg, L, pred_par[e->parent], pred_C[e->parent], h, nc->par, nc->C);
                }
                nc->chi2 = e->chi2;
                nc->hits[L] = e->hit;
                nc->n_hits = e->n_hits;
                if (log) ++log->n_update;
            } else if (e->kind == KIND_HOLE) {
                memcpy(nc->par, pred_par[e->parent], sizeof(nc->par));
                memcpy(nc->C, pred_C[e->parent], sizeof(nc->C));
                nc->n_holes++;
            }
        }
        memcpy(b->c, next, nn * sizeof(cand_t));
        b->n = nn;
    }
    free(ent);
}

static int same_outcome(const cand_t *a, const cand_t *b, int nl)
{
    if (a->status != b->status) return 0;
    for (int L = 0; L < nl; ++L)
        if (a->hits[L] != b->hits[L]) return 0;
    return 1;
}

static int cmp_decision(const void *va, const void *vb)
{
    const decision_t *a = (const decision_t *)va, *b = (const decision_t *)vb;
    /* in units of each kind's consideration window */
    const double ra = a->margin / (a->kind == 0 ? ORC_CUT_CONSIDER : ORC_RANK_CONSIDER);
    const double rb = b->margin / (b->kind == 0 ? ORC_CUT_CONSIDER : ORC_RANK_CONSIDER);
    return ra < rb ? -1 : (ra > rb ? 1 : 0);
}

/* re-runs per seed at most; decisions beyond count as relevant */
#define MAX_RERUNS 24

static void build_one(void *vctx, int64_t row)
{
    const build_ctx *bc = (const build_ctx *)vctx;
    const orc_config *cfg = bc->cfg;
    const int nl = cfg->n_layers, nsl = cfg->n_seed_layers;
    int k = cfg->max_cands;
    if (k > ORC_MAX_CANDS) k = ORC_MAX_CANDS;
    const int64_t sid = bc->seed_ids ? bc->seed_ids[row] : row;
    orc_track *o = &bc->out[row];

    beam_t b;
    memset(&b, 0, sizeof(b));
    b.n = 1;
    memcpy(b.c[0].par, bc->seed_par + 6 * sid, 6 * sizeof(double));
    unpack21(bc->seed_cov + 21 * sid, b.c[0].C);
    for (int L = 0; L < ORC_MAX_LAYERS; ++L) b.c[0].hits[L] = -1;
    for (int L = 0; L < nsl; ++L) {
        b.c[0].hits[L] = bc->seed_hits[sid * nsl + L];
        if (b.c[0].hits[L] >= 0) b.c[0].n_hits++;
    }

    run_log log;
    memset(&log, 0, sizeof(log));
    log.m_cut_raw = log.m_cut_far = log.m_rank_raw = log.m_rank_far = log.m_prop = INFINITY;
    log.snap = (beam_t *)malloc(ORC_MAX_LAYERS * sizeof(beam_t));
    run_layers(bc, nsl, &b, NULL, &log);

    if (b.n > 1 && b.c[0].n_hits == b.c[1].n_hits) {
        const double gap = (b.c[1].chi2 - b.c[0].chi2) / (1.0 + b.c[0].chi2);
        if (gap < log.m_rank_raw) log.m_rank_raw = gap;
        if (gap < ORC_RANK_CONSIDER) note_decision(&log, nl, -1, -1, 2, gap);
        else if (gap < log.m_rank_far) log.m_rank_far = gap;
    }

    /* which near decisions change the output: re-run each one inverted from
     * the beam before its layer, smallest margins first */
    double m_cut = log.m_cut_far, m_rank = log.m_rank_far;
    o->n_alt = 0;
    qsort(log.dec, log.n_dec, sizeof(decision_t), cmp_decision);
    for (int d = 0; d < log.n_dec; ++d) {
        const decision_t *dc = &log.dec[d];
        cand_t alt;
        int relevant = 1;
        if (dc->kind == 2) {
            alt = b.c[1];
        } else if (d < MAX_RERUNS) {
            beam_t rb = log.snap[dc->layer];
            run_layers(bc, dc->layer, &rb, dc, NULL);
            alt = rb.c[0];
            relevant = rb.n > 0 && !same_outcome(&alt, &b.c[0], nl);
        }
        if (!relevant) continue;
        if (dc->kind == 0) {
            if (dc->margin < m_cut) m_cut = dc->margin;
        } else if (dc->margin < m_rank) {
            m_rank = dc->margin;
        }
        if ((dc->kind == 2 || d < MAX_RERUNS) && o->n_alt < ORC_MAX_ALT) {
            const int a = o->n_alt++;
            o->alt_kind[a] = dc->kind;
            o->alt_margin[a] = dc->margin;
            for (int L = 0; L < ORC_MAX_LAYERS; ++L) o->alt_hits[a][L] = L < nl ? alt.hits[L] : -1;
            o->alt_status[a] = alt.status;
        }
    }
    free(log.dec);
    free(log.snap);

    const cand_t *best = &b.c[0];
    memcpy(o->par, best->par, sizeof(o->par));
    pack21(best->C, o->cov);
    o->chi2 = best->chi2;
    for (int L = 0; L < ORC_MAX_LAYERS; ++L) o->hits[L] = L < nl ? best->hits[L] : -1;
    o->n_hits = best->n_hits;
    o->n_holes = best->n_holes;
    o->status = best->status;
    o->n_final = b.n;
    o->m_cut = m_cut;
    o->m_rank = m_rank;
    o->m_prop = log.m_prop;
    o->m_cut_raw = log.m_cut_raw;
    o->m_rank_raw = log.m_rank_raw;
    o->n_prop = log.n_prop;
    o->n_accept = log.n_accept;
    o->n_update = log.n_update;
    if (bc->beam) {
        /* the whole final beam, rank by rank; ranks beyond it are empty (status -1) */
        for (int r = 0; r < k; ++r) {
            orc_track *t = &bc->beam[row * k + r];
            *t = *o;
            if (r >= b.n) {
                memset(t->par, 0, sizeof(t->par));
                memset(t->cov, 0, sizeof(t->cov));
                t->chi2 = 0.0;
                for (int L = 0; L < ORC_MAX_LAYERS; ++L) t->hits[L] = -1;
                t->n_hits = t->n_holes = 0;
                t->status = -1;
                continue;
            }
            const cand_t *cd = &b.c[r];
            memcpy(t->par, cd->par, sizeof(t->par));
            pack21(cd->C, t->cov);
            t->chi2 = cd->chi2;
            for (int L = 0; L < ORC_MAX_LAYERS; ++L) t->hits[L] = L < nl ? cd->hits[L] : -1;
            t->n_hits = cd->n_hits;
            t->n_holes = cd->n_holes;
            t->status = cd->status;
        }
    }
}

void orc_build(const orc_config *cfg, const orc_hits *hits, int32_t n_seeds_total,
               const double *seed_par, const double *seed_cov, const int32_t *seed_hits,
               const int32_t *seed_ids, int32_t n_sel, orc_track *out, int32_t n_threads)
{
    (void)n_seeds_total;
    build_ctx bc = {cfg, hits, seed_par, seed_cov, seed_hits, seed_ids, out, NULL};
    parallel_for(n_sel, n_threads, 4, build_one, &bc);
}

void orc_build_beam(const orc_config *cfg, const orc_hits *hits, int32_t n_seeds_total, const double *seed_par,
                    const double *seed_cov, const int32_t *seed_hits, const int32_t *seed_ids, int32_t n_sel,
                    orc_track *out, orc_track *beam, int32_t n_threads)
{
    (void)n_seeds_total;
    build_ctx bc = {cfg, hits, seed_par, seed_cov, seed_hits, seed_ids, out, beam};
    parallel_for(n_sel, n_threads, 4, build_one, &bc);
}

double orc_replay(const orc_config *cfg, const orc_hits *hits, const double seed_par[6],
                  const double seed_cov[21], const int32_t *layer_hits, double *layer_chi2,
                  int32_t *ok)
{
    double p[6], C[36], total = 0.0;
    memcpy(p, seed_par, sizeof(p));
    unpack21(seed_cov, C);
    *ok = 1;
    for (int L = 0; L < cfg->n_layers; ++L) layer_chi2[L] = -1.0;
    for (int L = cfg->n_seed_layers; L < cfg->n_layers; ++L) {
        double np[6], F[36];
        leave_layer(cfg, L - 1, p, C);
        if (to_layer(cfg, L, p, np, F, NULL)) {
            *ok = 0;
            break;
        }
        memcpy(p, np, sizeof(p));
        orc_transport(F, C);
        const int32_t h = layer_hits[L];
        if (h >= 0) {
            const double *hit = hits->xyz[L] + 3 * (int64_t)h;
            if (cfg->thick[L] > 0.0 && step_to_hit(cfg, L, p, C, hit, p, C)) {
                *ok = 0;
                break;
            }
            double c2 = layer_update(cfg, L, p, C, hit, p, C);
            layer_chi2[L] = c2;
            total += c2;
            if (!(c2 < cfg->chi2_cut)) *ok = 0;
        }
    }
    return total;
}
