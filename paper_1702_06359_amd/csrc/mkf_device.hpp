// FP32 device arithmetic of the Kalman filter: helix propagation with its
// Jacobian, covariance transport, multiple-scattering noise, hit chi2 and the
// measurement update.  One lane holds one track candidate; a state lives in
// registers as p[6] = (x, y, z, q/pT, phi, theta) and the symmetric
// covariance as its 21-entry packed upper triangle.
#pragma once

#include "mkf_internal.hpp"

namespace mkf {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kTwoPi = 6.28318530717958647692f;
constexpr float kInf = __builtin_huge_valf();

// index of element (i, j) of a symmetric 6x6 matrix in packed upper-triangle storage
__host__ __device__ constexpr int sym(int i, int j)
{
    return i <= j ? i * 6 - (i * (i - 1)) / 2 + (j - i) : j * 6 - (j * (j - 1)) / 2 + (i - j);
}

__device__ __forceinline__ float wrap_pi(float a)
{
    if (a > kPi) a -= kTwoPi;
    else if (a <= -kPi) a += kTwoPi;
    return a;
}

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Reads and writes through a pointer known to address global memory (global
// rather than flat instructions for pointers that were themselves loaded from
// memory; flat ones also count against the LDS wait counter).
__device__ __forceinline__ int load_global(const int *p)
{
    typedef const __attribute__((address_space(1))) int *gptr;
    return *(gptr)p;
}

__device__ __forceinline__ float load_global(const float *p)
{
    typedef const __attribute__((address_space(1))) float *gptr;
    return *(gptr)p;
}

__device__ __forceinline__ void store_global(float *p, float v)
{
    typedef __attribute__((address_space(1))) float *gptr;
    *(gptr)p = v;
}

__device__ __forceinline__ double load_global(const double *p)
{
    typedef const __attribute__((address_space(1))) double *gptr;
    return *(gptr)p;
}

__device__ __forceinline__ void store_global(double *p, double v)
{
    typedef __attribute__((address_space(1))) double *gptr;
    *(gptr)p = v;
}

__device__ __forceinline__ void store_global(int *p, int v)
{
    typedef __attribute__((address_space(1))) int *gptr;
    *(gptr)p = v;
}

__device__ __forceinline__ void store_global(float4 *p, float4 v)
{
    typedef float v4 __attribute__((ext_vector_type(4)));
    typedef __attribute__((address_space(1))) v4 *gptr;
    *(gptr)p = v4{v.x, v.y, v.z, v.w};
}

__device__ __forceinline__ void store_global(int4 *p, int4 v)
{
    typedef int v4 __attribute__((ext_vector_type(4)));
    typedef __attribute__((address_space(1))) v4 *gptr;
    *(gptr)p = v4{v.x, v.y, v.z, v.w};
}

__device__ __forceinline__ float4 load_global(const float4 *p)
{
    typedef float v4 __attribute__((ext_vector_type(4)));
    typedef const __attribute__((address_space(1))) v4 *gptr;
    const v4 v = *(gptr)p;
    return make_float4(v.x, v.y, v.z, v.w);
}

// An event descriptor as the kernels read it.  No kernel writes the
// descriptors, so they are read through the constant address space: with a
// wave-uniform event its fields become scalar loads into SGPRs, taken once,
// instead of vector loads that every global store would force the compiler
// to repeat.
typedef const __attribute__((address_space(4))) DevEvent CEvent;

__device__ __forceinline__ CEvent &event_desc(const DevEvent *events, int e) { return *(CEvent *)(events + e); }

// atan2 to 3.8e-7 rad: octant reduction and an odd degree-15 polynomial
// (least-squares fit to atan on [0, 1], max error 1.1e-7 in FP32; the
// rounding of results near pi dominates the total).  Used for the
// search-window centre, whose azimuth range is padded by 1e-5 rad, and for
// the azimuth bin of every hit (so a hit within that error of a bin edge may
// take either bin, and the padded window still covers it).
__device__ __forceinline__ float fast_atan2(float y, float x)
{
    const float ax = fabsf(x), ay = fabsf(y);
    const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
    const float t = mn * fast_rcp(mx);
    const float v = t * t;
    float r = fmaf(v, -0.00405456058f, 0.0218629526f);
    r = fmaf(v, r, -0.0559123558f);
    r = fmaf(v, r, 0.0964220321f);
    r = fmaf(v, r, -0.13908634f);
    r = fmaf(v, r, 0.199465672f);
    r = fmaf(v, r, -0.33329861f);
    r = fmaf(v, r, 0.999999336f);
    float a = t * r;
    if (ay > ax) a = 1.57079632679f - a;
    if (x < 0.f) a = 3.14159265359f - a;
    return copysignf(a, y);
}

// (sin, cos) of an angle advanced by a small increment d: series below
// |d| = 0.25 (error < 1e-9), the library sincos above.
__device__ __forceinline__ void rotate(float &s, float &c, float d)
{
    float sd, cd;
    if (fabsf(d) < 0.25f) {
        const float d2 = d * d;
        sd = d * fmaf(d2, fmaf(d2, fmaf(d2, -1.f / 5040.f, 1.f / 120.f), -1.f / 6.f), 1.f);
        cd = fmaf(d2, fmaf(d2, fmaf(d2, -1.f / 720.f, 1.f / 24.f), -0.5f), 1.f);
    } else {
        sincosf(d, &sd, &cd);
    }
    const float ns = fmaf(s, cd, c * sd);
    c = fmaf(c, cd, -s * sd);
    s = ns;
}

// Structure of the propagation Jacobian in (x, y, z, q/pT, phi, theta):
// 0 = known zero, 2 = known one, 1 = computed.  The transport below is
// unrolled against this pattern so known zeros and ones cost nothing (the
// paper's Matriplex generator does the same for its CPU kernels, Section 2.1).
// To a cylinder the path depends on the transverse inputs; to a plane of
// fixed z it depends on z and theta only, and z leaves with no variance.
constexpr signed char kFpatCyl[6][6] = {
    {1, 1, 0, 1, 1, 0},
    {1, 1, 0, 1, 1, 0},
    {1, 1, 2, 1, 1, 1},
    {0, 0, 0, 2, 0, 0},
    {1, 1, 0, 1, 1, 0},
    {0, 0, 0, 0, 0, 2},
};
constexpr signed char kFpatDisk[6][6] = {
    {2, 0, 1, 1, 1, 1},
    {0, 2, 1, 1, 1, 1},
    {0, 0, 0, 0, 0, 0},
    {0, 0, 0, 2, 0, 0},
    {0, 0, 1, 1, 2, 1},
    {0, 0, 0, 0, 0, 2},
};

// C <- F C F^T on the packed covariance, F of a cylinder (kDisk false) or a
// disk crossing.
template <bool kDisk>
__device__ __forceinline__ void transport(const float (&F)[6][6], float (&c)[21])
{
    constexpr const signed char(&kFpat)[6][6] = kDisk ? kFpatDisk : kFpatCyl;
    float M[6][6];   // F C
#pragma unroll
    for (int i = 0; i < 6; ++i) {
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            float acc = 0.f;
            bool first = true;
#pragma unroll
            for (int t = 0; t < 6; ++t) {
                if (kFpat[i][t] == 0) continue;
                const float v = c[sym(t, j)];
                if (first) acc = (kFpat[i][t] == 2) ? v : F[i][t] * v;
                else acc = (kFpat[i][t] == 2) ? acc + v : fmaf(F[i][t], v, acc);
                first = false;
            }
            M[i][j] = acc;
        }
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) {
#pragma unroll
        for (int k = i; k < 6; ++k) {
            float acc = 0.f;
            bool first = true;
#pragma unroll
            for (int t = 0; t < 6; ++t) {
                if (kFpat[k][t] == 0) continue;
                const float v = M[i][t];
                if (first) acc = (kFpat[k][t] == 2) ? v : v * F[k][t];
                else acc = (kFpat[k][t] == 2) ? acc + v : fmaf(v, F[k][t], acc);
                first = false;
            }
            c[sym(i, k)] = acc;
        }
    }
}

// Position block of F C F^T only (xx, xy, yy, xz, yz, zz): what the chi2 of
// a hit needs after the second step of a thick layer.
template <bool kDisk>
__device__ __forceinline__ void transport_pos(const float (&F)[6][6], const float (&c)[21], float (&cp)[6])
{
    constexpr const signed char(&kFpat)[6][6] = kDisk ? kFpatDisk : kFpatCyl;
    float M[3][6];   // rows 0..2 of F C
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            float acc = 0.f;
            bool first = true;
#pragma unroll
            for (int t = 0; t < 6; ++t) {
                if (kFpat[i][t] == 0) continue;
                const float v = c[sym(t, j)];
                if (first) acc = (kFpat[i][t] == 2) ? v : F[i][t] * v;
                else acc = (kFpat[i][t] == 2) ? acc + v : fmaf(F[i][t], v, acc);
                first = false;
            }
            M[i][j] = acc;
        }
    }
    constexpr int kI[6] = {0, 0, 1, 0, 1, 2}, kK[6] = {0, 1, 1, 2, 2, 2};
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        const int i = kI[e], k = kK[e];
        float acc = 0.f;
        bool first = true;
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            if (kFpat[k][t] == 0) continue;
            const float v = M[i][t];
            if (first) acc = (kFpat[k][t] == 2) ? v : v * F[k][t];
            else acc = (kFpat[k][t] == 2) ? acc + v : fmaf(v, F[k][t], acc);
            first = false;
        }
        cp[e] = acc;
    }
}

// sin(a)/a, (1-cos a)/a and their derivatives (a cos a - sin a)/a^2,
// (a sin a - 1 + cos a)/a^2: series below |a| = 0.5, where the direct forms
// lose FP32 digits to cancellation.
__device__ __forceinline__ void turn_terms(float a, float &S1, float &C1, float &S2, float &C2)
{
    if (fabsf(a) < 0.5f) {
        const float a2 = a * a;
        S1 = fmaf(a2, fmaf(a2, fmaf(a2, fmaf(a2, 1.f / 362880.f, -1.f / 5040.f), 1.f / 120.f), -1.f / 6.f), 1.f);
        C1 = a * fmaf(a2, fmaf(a2, fmaf(a2, fmaf(a2, 1.f / 3628800.f, -1.f / 40320.f), 1.f / 720.f), -1.f / 24.f), 0.5f);
        S2 = a * fmaf(a2, fmaf(a2, fmaf(a2, 1.f / 45360.f, -1.f / 840.f), 1.f / 30.f), -1.f / 3.f);
        C2 = fmaf(a2, fmaf(a2, fmaf(a2, fmaf(a2, 1.f / 403200.f, -1.f / 5760.f), 1.f / 144.f), -0.125f), 0.5f);
    } else {
        float sa, ca;
        sincosf(a, &sa, &ca);
        const float ia = fast_rcp(a);
        S1 = sa * ia;
        C1 = (1.f - ca) * ia;
        S2 = (a * ca - sa) * ia * ia;
        C2 = (a * sa - 1.f + ca) * ia * ia;
    }
}

// atan(u)/u: series below |u| = 0.25 (error < 1e-9), the library atan above
__device__ __forceinline__ float atanc(float u)
{
    if (fabsf(u) < 0.25f) {
        const float v = u * u;
        // 1 - v/3 + v^2/5 - v^3/7 + v^4/9 - v^5/11 + v^6/13
        float r = fmaf(v, 1.f / 13.f, -1.f / 11.f);
        r = fmaf(v, r, 1.f / 9.f);
        r = fmaf(v, r, -1.f / 7.f);
        r = fmaf(v, r, 1.f / 5.f);
        r = fmaf(v, r, -1.f / 3.f);
        return fmaf(v, r, 1.f);
    }
    return atanf(u) * fast_rcp(u);
}

// sines and cosines of the momentum angles of a state
struct Trig {
    float sph, cph, sth, cth;
};

__device__ __forceinline__ Trig trig_of(const float (&p)[6])
{
    Trig t;
    sincosf(p[4], &t.sph, &t.cph);
    sincosf(p[5], &t.sth, &t.cth);
    return t;
}

// Jacobian of a step to a cylinder in factored form, F = P + v d^T: P the
// derivative at fixed path (the identity but for six entries), v the
// derivative of the end point (x, y, z, phi) along the transverse path, and
// d the change of path with (x, y, q/pT, phi) that keeps the end point on the
// cylinder.  Rows q/pT and theta are those of the identity.
struct CylJac {
    float Pxq, Pxp, Pyq, Pyp, Pzt, Ppq;   // P[0][3], P[0][4], P[1][3], P[1][4], P[2][5], P[4][3]
    float vx, vy, vz, vp;                 // v[0], v[1], v[2], v[4]
    float dx, dy, dq, dp;                 // d[0], d[1], d[3], d[4]
};

__device__ __forceinline__ void helix_cyl(const float (&p)[6], const Trig &tg, float s, float w_per_qpt,
                                          float (&o)[6], CylJac &J, float &sn_out, float &cn_out);

// The full 6x6 matrix of a factored cylinder Jacobian.
__device__ __forceinline__ void cyl_jac_full(const CylJac &J, float (&F)[6][6])
{
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < 6; ++j) F[i][j] = i == j ? 1.f : 0.f;
    const float v[4] = {J.vx, J.vy, J.vz, J.vp};
    const int row[4] = {0, 1, 2, 4};
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        F[row[a]][0] = fmaf(v[a], J.dx, F[row[a]][0]);
        F[row[a]][1] = fmaf(v[a], J.dy, F[row[a]][1]);
        F[row[a]][3] = fmaf(v[a], J.dq, F[row[a]][3]);
        F[row[a]][4] = fmaf(v[a], J.dp, F[row[a]][4]);
    }
    F[0][3] += J.Pxq;
    F[0][4] += J.Pxp;
    F[1][3] += J.Pyq;
    F[1][4] += J.Pyp;
    F[2][5] = J.Pzt;
    F[4][3] += J.Ppq;
}

// C <- F C F^T for a factored cylinder Jacobian F = P + v d^T:
// P C P^T + (P u) v^T + v (P u)^T + (d^T u) v v^T with u = C d, about 110
// multiply-adds where the general sparse product takes about 170.
__device__ __forceinline__ void transport_cyl(const CylJac &J, float (&c)[21])
{
    auto C = [&](int i, int j) { return c[sym(i, j)]; };
    float u[6];
#pragma unroll
    for (int i = 0; i < 6; ++i)
        u[i] = fmaf(C(i, 0), J.dx, fmaf(C(i, 1), J.dy, fmaf(C(i, 3), J.dq, C(i, 4) * J.dp)));
    const float sig = fmaf(J.dx, u[0], fmaf(J.dy, u[1], fmaf(J.dq, u[3], J.dp * u[4])));
    float Pu[6];
    Pu[0] = fmaf(J.Pxq, u[3], fmaf(J.Pxp, u[4], u[0]));
    Pu[1] = fmaf(J.Pyq, u[3], fmaf(J.Pyp, u[4], u[1]));
    Pu[2] = fmaf(J.Pzt, u[5], u[2]);
    Pu[3] = u[3];
    Pu[4] = fmaf(J.Ppq, u[3], u[4]);
    Pu[5] = u[5];
    // M = P C: the entries the upper triangle of M P^T needs
    auto M = [&](int i, int j) {
        switch (i) {
        case 0: return fmaf(J.Pxq, C(3, j), fmaf(J.Pxp, C(4, j), C(0, j)));
        case 1: return fmaf(J.Pyq, C(3, j), fmaf(J.Pyp, C(4, j), C(1, j)));
        case 2: return fmaf(J.Pzt, C(5, j), C(2, j));
        case 4: return fmaf(J.Ppq, C(3, j), C(4, j));
        default: return C(i, j);
        }
    };
    float M3[5], M4[5], M5[6];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        M3[i] = M(i, 3);
        M4[i] = M(i, 4);
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) M5[i] = M(i, 5);
    float n[21];
    // column k of N = M P^T for i <= k
    n[sym(0, 0)] = fmaf(J.Pxq, M3[0], fmaf(J.Pxp, M4[0], M(0, 0)));
#pragma unroll
    for (int i = 0; i < 2; ++i) n[sym(i, 1)] = fmaf(J.Pyq, M3[i], fmaf(J.Pyp, M4[i], M(i, 1)));
#pragma unroll
    for (int i = 0; i < 3; ++i) n[sym(i, 2)] = fmaf(J.Pzt, M5[i], M(i, 2));
#pragma unroll
    for (int i = 0; i < 4; ++i) n[sym(i, 3)] = M3[i];
#pragma unroll
    for (int i = 0; i < 5; ++i) n[sym(i, 4)] = fmaf(J.Ppq, M3[i], M4[i]);
#pragma unroll
    for (int i = 0; i < 6; ++i) n[sym(i, 5)] = M5[i];
    // + (P u) v^T + v (P u)^T + sig v v^T, v nonzero in rows 0, 1, 2, 4
    const float v[6] = {J.vx, J.vy, J.vz, 0.f, J.vp, 0.f};
    constexpr bool inV[6] = {true, true, true, false, true, false};
    const float hs = 0.5f * sig;
    float t[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) t[i] = inV[i] ? fmaf(hs, v[i], Pu[i]) : Pu[i];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
#pragma unroll
        for (int k = i; k < 6; ++k) {
            float a = n[sym(i, k)];
            if (inV[i] && inV[k]) a = fmaf(t[i], v[k], fmaf(v[i], t[k], a));
            else if (inV[i]) a = fmaf(v[i], Pu[k], a);
            else if (inV[k]) a = fmaf(Pu[i], v[k], a);
            c[sym(i, k)] = a;
        }
    }
}

// Propagate state p (with the sines and cosines of its angles in tg) to the
// cylinder of radius r along the helix of the
// uniform field (curvature w = w_per_qpt * q/pT, w > 0 turning
// counter-clockwise).  The transverse path s is the smallest positive root of
// the half-turn-angle quadratic  alpha T^2 + b T - D/4 = 0  (T = tan(a/2)/w,
// a = w s) of the chord condition |(x,y) + chord| = r; its w -> 0 limit is the
// straight line.  Writes the new state o and the Jacobian F = d o / d p on
// the cylinder (the derivative at fixed s plus the change of s that keeps the
// end point on the cylinder), and the sine and cosine of the new momentum
// azimuth.  Returns false when r is never reached.
__device__ __forceinline__ bool propagate(const float (&p)[6], const Trig &tg, float r, float w_per_qpt,
                                          float (&o)[6], CylJac &J, float &sn_out, float &cn_out)
{
    const float x = p[0], y = p[1], q = p[3];
    const float sph = tg.sph, cph = tg.cph;
    const float w = w_per_qpt * q;
    const float b = fmaf(x, cph, y * sph);
    const float e = fmaf(y, cph, -x * sph);
    const float D = fmaf(r, r, -fmaf(x, x, y * y));
    const float alpha = fmaf(w, e, 1.f) - 0.25f * w * w * D;
    const float disc = fmaf(b, b, alpha * D);
    if (!(disc >= 0.f)) return false;
    const float qd = __builtin_amdgcn_sqrtf(disc);
    const float smin = 1e-6f * r;
    // near-half root: when valid it is the first crossing, since every
    // far-half solution is longer than pi/|w|
    const float T1 = (b + qd != 0.f) ? 0.5f * D * fast_rcp(b + qd) : kInf;
    float s = (fabsf(T1) < kInf) ? 2.f * T1 * atanc(w * T1) : -1.f;
    if (!(s > smin && s * fabsf(w) <= kPi)) {
        s = kInf;
        const float roots[2] = {T1, (alpha != 0.f) ? -(b + qd) / (2.f * alpha) : kInf};
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const float T = roots[i];
            if (!(fabsf(T) < kInf)) continue;
            const float u = w * T;
            const float s1 = 2.f * T * atanc(u);
            if (s1 > smin && s1 < s) s = s1;
            if (w != 0.f) {
                const float s2 = 2.f * (atanf(u) + copysignf(kPi, w)) / w;
                if (s2 > smin && s2 < s) s = s2;
            }
        }
        if (!(s < kInf)) return false;
    }
    helix_cyl(p, tg, s, w_per_qpt, o, J, sn_out, cn_out);
    return true;
}

// The helix step of transverse path s (either sign) from state p, and the
// Jacobian on the cylinder through the end point (see propagate).
__device__ __forceinline__ void helix_cyl(const float (&p)[6], const Trig &tg, float s, float w_per_qpt,
                                          float (&o)[6], CylJac &J, float &sn_out, float &cn_out)
{
    const float x = p[0], y = p[1], z = p[2], q = p[3], phi = p[4];
    const float sph = tg.sph, cph = tg.cph;
    const float w = w_per_qpt * q;
    const float a = w * s;
    float S1, C1, S2, C2;
    turn_terms(a, S1, C1, S2, C2);
    const float A = fmaf(cph, S1, -sph * C1);     // (sin(phi+a) - sin phi)/a
    const float B = fmaf(cph, C1, sph * S1);      // (cos phi - cos(phi+a))/a
    const float gx = fmaf(cph, S2, -sph * C2);    // dA/da
    const float gy = fmaf(sph, S2, cph * C2);     // dB/da
    const float ist = fast_rcp(tg.sth);
    const float cot = tg.cth * ist;
    const float nx = fmaf(s, A, x), ny = fmaf(s, B, y);
    const float ca = fmaf(-a, C1, 1.f), sa = a * S1;       // cos a, sin a
    const float cn = fmaf(cph, ca, -sph * sa), sn = fmaf(sph, ca, cph * sa);
    o[0] = nx;
    o[1] = ny;
    o[2] = fmaf(s, cot, z);
    o[3] = q;
    o[4] = wrap_pi(phi + a);
    o[5] = p[5];
    sn_out = sn;
    cn_out = cn;

    // derivatives at fixed path
    const float Pxq = s * s * gx * w_per_qpt, Pxp = -s * B;
    const float Pyq = s * s * gy * w_per_qpt, Pyp = s * A;
    const float Pzt = -s * ist * ist;
    const float Ppq = s * w_per_qpt;
    // d s / d p from x'^2 + y'^2 = r^2
    const float iden = -fast_rcp(fmaf(nx, cn, ny * sn));
    const float dsx = nx * iden, dsy = ny * iden;
    const float dsq = fmaf(nx, Pxq, ny * Pyq) * iden;
    const float dsp = fmaf(nx, Pxp, ny * Pyp) * iden;
    J = CylJac{Pxq, Pxp, Pyq, Pyp, Pzt, Ppq, cn, sn, cot, w, dsx, dsy, dsq, dsp};
}

// Second step of the two-step propagation on a layer of finite thickness:
// from the layer's average cylinder to the nearby cylinder of radius r
// through a hit, ahead or behind.  Of the two roots of the path quadratic
// (principal branch) the one of smaller |s|.  False when r is never reached;
// o and F are then those of a zero step, so callers may use them unguarded.
__device__ __forceinline__ bool step_near_cyl(const float (&p)[6], const Trig &tg, float r, float w_per_qpt,
                                              float (&o)[6], float (&F)[6][6], float &sn_out, float &cn_out)
{
    const float x = p[0], y = p[1];
    const float w = w_per_qpt * p[3];
    const float b = fmaf(x, tg.cph, y * tg.sph);
    const float e = fmaf(y, tg.cph, -x * tg.sph);
    const float D = fmaf(r, r, -fmaf(x, x, y * y));
    const float alpha = fmaf(w, e, 1.f) - 0.25f * w * w * D;
    const float disc = fmaf(b, b, alpha * D);
    bool ok = disc >= 0.f;
    const float qd = __builtin_amdgcn_sqrtf(fmaxf(disc, 0.f));
    const float bq = b >= 0.f ? b + qd : b - qd;
    float s = 0.f;
    if (bq != 0.f) {
        const float T1 = 0.5f * D / bq;
        s = 2.f * T1 * atanc(w * T1);
        if (alpha != 0.f) {
            const float T2 = -0.5f * bq / alpha;
            const float s2 = 2.f * T2 * atanc(w * T2);
            if (fabsf(s2) < fabsf(s)) s = s2;
        }
    } else if (D != 0.f) {
        ok = false;
    }
    if (!ok || !(fabsf(s) < kInf)) {
        ok = false;
        s = 0.f;
    }
    CylJac J;
    helix_cyl(p, tg, s, w_per_qpt, o, J, sn_out, cn_out);
    cyl_jac_full(J, F);
    return ok;
}

__device__ __forceinline__ void helix_plane(const float (&p)[6], const Trig &tg, float s, float zd, float w_per_qpt,
                                            float (&o)[6], float (&F)[6][6], float &sn_out, float &cn_out);

// Propagate state p to the plane z = zd (an endcap disk): the transverse
// path is fixed by the dip angle, s = (zd - z) tan(theta), and must be
// positive (the helix heads towards the plane).  Same helix and outputs as
// propagate(); the Jacobian's path term keeps z on the plane, so it depends
// on z and theta only and the z row vanishes.
__device__ __forceinline__ bool propagate_plane(const float (&p)[6], const Trig &tg, float zd, float w_per_qpt,
                                                float (&o)[6], float (&F)[6][6], float &sn_out, float &cn_out)
{
    const float s = (zd - p[2]) * (tg.sth * fast_rcp(tg.cth));
    if (!(s > 0.f) || !(s < kInf)) return false;
    helix_plane(p, tg, s, zd, w_per_qpt, o, F, sn_out, cn_out);
    return true;
}

// The helix step of transverse path s (either sign) from state p onto the
// plane z = zd, and the Jacobian on that plane (see propagate_plane).
__device__ __forceinline__ void helix_plane(const float (&p)[6], const Trig &tg, float s, float zd, float w_per_qpt,
                                            float (&o)[6], float (&F)[6][6], float &sn_out, float &cn_out)
{
    const float x = p[0], y = p[1], q = p[3], phi = p[4];
    const float sph = tg.sph, cph = tg.cph;
    const float w = w_per_qpt * q;
    const float ict = fast_rcp(tg.cth);
    const float tanth = tg.sth * ict;
    const float a = w * s;
    float S1, C1, S2, C2;
    turn_terms(a, S1, C1, S2, C2);
    const float A = fmaf(cph, S1, -sph * C1);
    const float B = fmaf(cph, C1, sph * S1);
    const float gx = fmaf(cph, S2, -sph * C2);
    const float gy = fmaf(sph, S2, cph * C2);
    const float ca = fmaf(-a, C1, 1.f), sa = a * S1;
    const float cn = fmaf(cph, ca, -sph * sa), sn = fmaf(sph, ca, cph * sa);
    o[0] = fmaf(s, A, x);
    o[1] = fmaf(s, B, y);
    o[2] = zd;
    o[3] = q;
    o[4] = wrap_pi(phi + a);
    o[5] = p[5];
    sn_out = sn;
    cn_out = cn;

    // derivatives at fixed path, plus d s / d(z, theta) = (-tan theta,
    // s / (sin theta cos theta)) from z + s cot(theta) = zd
    const float Pxq = s * s * gx * w_per_qpt, Pxp = -s * B;
    const float Pyq = s * s * gy * w_per_qpt, Pyp = s * A;
    const float Ppq = s * w_per_qpt;
    const float dsz = -tanth;
    const float dst = s * ict * fast_rcp(tg.sth);
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < 6; ++j) F[i][j] = 0.f;
    F[0][0] = 1.f;
    F[0][2] = cn * dsz;
    F[0][3] = Pxq;
    F[0][4] = Pxp;
    F[0][5] = cn * dst;
    F[1][1] = 1.f;
    F[1][2] = sn * dsz;
    F[1][3] = Pyq;
    F[1][4] = Pyp;
    F[1][5] = sn * dst;
    F[3][3] = 1.f;
    F[4][2] = w * dsz;
    F[4][3] = Ppq;
    F[4][4] = 1.f;
    F[4][5] = w * dst;
    F[5][5] = 1.f;
}

// Second step onto the plane z = zd through a hit of a thick disk, ahead or
// behind: s = (zd - z) tan(theta) of either sign.
__device__ __forceinline__ bool step_near_plane(const float (&p)[6], const Trig &tg, float zd, float w_per_qpt,
                                                float (&o)[6], float (&F)[6][6], float &sn_out, float &cn_out)
{
    float s = (zd - p[2]) * (tg.sth * fast_rcp(tg.cth));
    const bool ok = fabsf(s) < kInf;
    if (!ok) s = 0.f;   // a zero step: o and F stay defined
    helix_plane(p, tg, s, zd, w_per_qpt, o, F, sn_out, cn_out);
    return ok;
}

// Multiple scattering in a layer of x0 radiation lengths, crossed at the
// state's position: Highland angle th0 with the path factor 1/|cos alpha|
// (alpha to the layer normal: radial on a cylinder, z on a disk), added to
// (q/pT, phi, theta) at fixed |p|.
__device__ __forceinline__ void add_scattering(const float (&p)[6], const Trig &tg, float x0, bool disk,
                                               float mass2, float (&c)[21])
{
    if (!(x0 > 0.f)) return;
    const float x = p[0], y = p[1], q = p[3];
    const float ir0 = __builtin_amdgcn_rsqf(fmaf(x, x, y * y));
    const float cosa = disk ? fmaxf(fabsf(tg.cth), 1e-6f)
                            : fmaxf(fabsf(tg.sth * fmaf(tg.cph, x * ir0, tg.sph * y * ir0)), 1e-6f);
    const float t = x0 * fast_rcp(cosa);
    const float k = fabsf(q) * tg.sth;                                          // 1/|p|
    const float inv_bp = k * __builtin_amdgcn_sqrtf(fmaf(mass2 * k, k, 1.f));    // 1/(beta p)
    const float th0 = 0.0136f * inv_bp * __builtin_amdgcn_sqrtf(t) * fmaf(0.038f, __logf(t), 1.f);
    const float v = th0 * th0;
    const float ist = fast_rcp(tg.sth);
    const float cot = tg.cth * ist;
    c[sym(4, 4)] += v * ist * ist;
    c[sym(5, 5)] += v;
    c[sym(3, 3)] += q * q * cot * cot * v;
    c[sym(3, 5)] -= q * cot * v;
}

// Prediction on the next surface (Section 2: propagate, then add the
// scattering of the layer left, then transport the covariance): the state
// np with the sine and cosine of its azimuth, the covariance c updated in
// place.  False when the helix never reaches the surface (c untouched).
template <bool kDisk>
__device__ __forceinline__ bool predict(const float (&p)[6], const Trig &tg, float where, float w_per_qpt, float x0,
                                        float mass2, float (&np)[6], float &sn, float &cn, float (&c)[21])
{
    if constexpr (kDisk) {
        float F[6][6];
        if (!propagate_plane(p, tg, where, w_per_qpt, np, F, sn, cn)) return false;
        add_scattering(p, tg, x0, true, mass2, c);
        transport<true>(F, c);
    } else {
        CylJac J;
        if (!propagate(p, tg, where, w_per_qpt, np, J, sn, cn)) return false;
        add_scattering(p, tg, x0, false, mass2, c);
        transport_cyl(J, c);
    }
    return true;
}

// chi2 of a hit (cos phi_h, sin phi_h, z_h) against a predicted state: the
// residual on the plane tangent to the layer at the hit, u along
// (-sin phi_h, cos phi_h, 0) and z, with S = H C H^T + V.
__device__ __forceinline__ float hit_chi2(float x, float y, float z, float cxx, float cxy, float cyy, float cxz,
                                          float cyz, float czz, float ch, float sh, float zh, float var_u,
                                          float var_z)
{
    const float ru = fmaf(x, sh, -y * ch);
    const float rz = zh - z;
    const float suu = fmaf(sh * sh, cxx, fmaf(-2.f * sh * ch, cxy, fmaf(ch * ch, cyy, var_u)));
    const float suz = fmaf(-sh, cxz, ch * cyz);
    const float szz = czz + var_z;
    const float idet = fast_rcp(fmaf(suu, szz, -suz * suz));
    return fmaf(szz * ru, ru, fmaf(-2.f * suz * ru, rz, suu * rz * rz)) * idet;
}

// chi2 of a disk hit (cos phi_h, sin phi_h, r_h) against a predicted state
// on the disk's plane: residuals u along (-sin phi_h, cos phi_h) and v along
// (cos phi_h, sin phi_h), S = H C H^T + diag(var_u, var_r).
__device__ __forceinline__ float hit_chi2_disk(float x, float y, float cxx, float cxy, float cyy, float ch, float sh,
                                               float rh, float var_u, float var_r)
{
    const float ru = fmaf(x, sh, -y * ch);
    const float rv = rh - fmaf(x, ch, y * sh);
    const float sc2 = 2.f * sh * ch;
    const float ss = sh * sh, cc = ch * ch;
    const float suu = fmaf(ss, cxx, fmaf(-sc2, cxy, fmaf(cc, cyy, var_u)));
    const float svv = fmaf(cc, cxx, fmaf(sc2, cxy, fmaf(ss, cyy, var_r)));
    const float suv = fmaf(0.5f * sc2, cyy - cxx, (cc - ss) * cxy);
    const float idet = fast_rcp(fmaf(suu, svv, -suv * suv));
    return fmaf(svv * ru, ru, fmaf(-2.f * suv * ru, rv, suu * rv * rv)) * idet;
}

// Kalman update with one hit.  K = C H^T S^-1, p += K r, C -= K (H C) on the
// upper triangle (so C stays exactly symmetric).  Returns the hit's chi2.
// The first measured coordinate is u along (-sin phi_h, cos phi_h, 0); the
// second (value zh) is z on a cylinder, r along (cos phi_h, sin phi_h, 0) on
// a disk (kDisk), with variance var_z.
template <bool kDisk>
__device__ __forceinline__ float kf_update(float (&p)[6], float (&c)[21], Trig &tg, float ch, float sh, float zh,
                                           float var_u, float var_z)
{
    const float ru = fmaf(p[0], sh, -p[1] * ch);
    const float rz = kDisk ? zh - fmaf(p[0], ch, p[1] * sh) : zh - p[2];
    float Mu[6], Mz[6];   // rows of H C
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        Mu[j] = fmaf(-sh, c[sym(0, j)], ch * c[sym(1, j)]);
        Mz[j] = kDisk ? fmaf(ch, c[sym(0, j)], sh * c[sym(1, j)]) : c[sym(2, j)];
    }
    const float suu = fmaf(-sh, Mu[0], fmaf(ch, Mu[1], var_u));
    const float suz = kDisk ? fmaf(ch, Mu[0], sh * Mu[1]) : Mu[2];
    const float szz = kDisk ? fmaf(ch, Mz[0], fmaf(sh, Mz[1], var_z)) : Mz[2] + var_z;
    const float idet = fast_rcp(fmaf(suu, szz, -suz * suz));
    const float i00 = szz * idet, i01 = -suz * idet, i11 = suu * idet;
    const float chi2 = fmaf(ru, fmaf(i00, ru, i01 * rz), rz * fmaf(i01, ru, i11 * rz));
    float K0[6], K1[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        K0[j] = fmaf(Mu[j], i00, Mz[j] * i01);
        K1[j] = fmaf(Mu[j], i01, Mz[j] * i11);
    }
    float dp[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        dp[j] = fmaf(K0[j], ru, K1[j] * rz);
        p[j] += dp[j];
    }
    p[4] = wrap_pi(p[4]);
    rotate(tg.sph, tg.cph, dp[4]);
    rotate(tg.sth, tg.cth, dp[5]);
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i; j < 6; ++j) c[sym(i, j)] -= fmaf(K0[i], Mu[j], K1[i] * Mz[j]);
    return chi2;
}

// Kalman update in Joseph form, C' = (I - K H) C (I - K H)^T + K V K^T.
// Used where the prediction is much looser than the hit (a fit starting
// from a wide prior): there C - K H C subtracts two nearly equal numbers and
// loses FP32 digits, while the Joseph form only scales them by (I - K H).
// Measured coordinates as in kf_update.
template <bool kDisk>
__device__ __forceinline__ float kf_update_joseph(float (&p)[6], float (&c)[21], Trig &tg, float ch, float sh,
                                                  float zh, float var_u, float var_z)
{
    const float ru = fmaf(p[0], sh, -p[1] * ch);
    const float rz = kDisk ? zh - fmaf(p[0], ch, p[1] * sh) : zh - p[2];
    float Mu[6], Mz[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        Mu[j] = fmaf(-sh, c[sym(0, j)], ch * c[sym(1, j)]);
        Mz[j] = kDisk ? fmaf(ch, c[sym(0, j)], sh * c[sym(1, j)]) : c[sym(2, j)];
    }
    const float suu = fmaf(-sh, Mu[0], fmaf(ch, Mu[1], var_u));
    const float suz = kDisk ? fmaf(ch, Mu[0], sh * Mu[1]) : Mu[2];
    const float szz = kDisk ? fmaf(ch, Mz[0], fmaf(sh, Mz[1], var_z)) : Mz[2] + var_z;
    const float idet = 1.f / fmaf(suu, szz, -suz * suz);
    const float i00 = szz * idet, i01 = -suz * idet, i11 = suu * idet;
    const float chi2 = fmaf(ru, fmaf(i00, ru, i01 * rz), rz * fmaf(i01, ru, i11 * rz));
    float K0[6], K1[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        K0[j] = fmaf(Mu[j], i00, Mz[j] * i01);
        K1[j] = fmaf(Mu[j], i01, Mz[j] * i11);
    }
    float dp[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        dp[j] = fmaf(K0[j], ru, K1[j] * rz);
        p[j] += dp[j];
    }
    p[4] = wrap_pi(p[4]);
    rotate(tg.sph, tg.cph, dp[4]);
    rotate(tg.sth, tg.cth, dp[5]);
    // one row of D = (I - K H) C at a time; the result goes to a fresh array
    // because every row of D reads the old C
    float nc[21];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        float D[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) D[j] = c[sym(i, j)] - fmaf(K0[i], Mu[j], K1[i] * Mz[j]);
        const float du = fmaf(-sh, D[0], ch * D[1]);                    // (D H^T)_iu
        const float dz = kDisk ? fmaf(ch, D[0], sh * D[1]) : D[2];      // (D H^T)_i2
#pragma unroll
        for (int j = i; j < 6; ++j) {
            const float kvk = fmaf(var_u * K0[i], K0[j], var_z * K1[i] * K1[j]);
            nc[sym(i, j)] = D[j] - fmaf(du, K0[j], dz * K1[j]) + kvk;
        }
    }
#pragma unroll
    for (int i = 0; i < 21; ++i) c[i] = nc[i];
    return chi2;
}

// ---- 3x3 global-Cartesian measurement ----------------------------------------
// The hit's position (x, y, z) measured with the error ellipsoid
// V = var_u u u^T + var_r n n^T + var_z e_z e_z^T (u = (-sin, cos, 0) and
// n = (cos, sin, 0) at the hit's azimuth); H = [I3 0].

struct Sym3 {           // symmetric 3x3: xx, xy, yy, xz, yz, zz
    float a[6];
};

__device__ __forceinline__ Sym3 hit_ellipsoid(float ch, float sh, float var_u, float var_r, float var_z)
{
    Sym3 v;
    v.a[0] = fmaf(var_u * sh, sh, var_r * ch * ch);
    v.a[1] = (var_r - var_u) * sh * ch;
    v.a[2] = fmaf(var_u * ch, ch, var_r * sh * sh);
    v.a[3] = 0.f;
    v.a[4] = 0.f;
    v.a[5] = var_z;
    return v;
}

// inverse of a symmetric 3x3 by its cofactors
__device__ __forceinline__ Sym3 inverse_sym3(const Sym3 &s)
{
    const float xx = s.a[0], xy = s.a[1], yy = s.a[2], xz = s.a[3], yz = s.a[4], zz = s.a[5];
    Sym3 b;
    b.a[0] = fmaf(yy, zz, -yz * yz);
    b.a[1] = fmaf(xz, yz, -xy * zz);
    b.a[2] = fmaf(xx, zz, -xz * xz);
    b.a[3] = fmaf(xy, yz, -xz * yy);
    b.a[4] = fmaf(xy, xz, -xx * yz);
    b.a[5] = fmaf(xx, yy, -xy * xy);
    const float idet = 1.f / fmaf(xx, b.a[0], fmaf(xy, b.a[1], xz * b.a[3]));
#pragma unroll
    for (int i = 0; i < 6; ++i) b.a[i] *= idet;
    return b;
}

__device__ __forceinline__ constexpr int s3(int i, int j)
{
    return i == j ? (i == 0 ? 0 : (i == 1 ? 2 : 5)) : ((i + j) == 1 ? 1 : ((i + j) == 2 ? 3 : 4));
}

// chi2 of a hit (hx, hy, hz) against a predicted position with covariance
// (cxx, cxy, cyy, cxz, cyz, czz)
__device__ __forceinline__ float hit_chi2_3d(float x, float y, float z, float cxx, float cxy, float cyy, float cxz,
                                             float cyz, float czz, float hx, float hy, float hz, float var_u,
                                             float var_r, float var_z)
{
    const float irh = __builtin_amdgcn_rsqf(fmaf(hx, hx, hy * hy));
    const Sym3 v = hit_ellipsoid(hx * irh, hy * irh, var_u, var_r, var_z);
    Sym3 S;
    S.a[0] = cxx + v.a[0];
    S.a[1] = cxy + v.a[1];
    S.a[2] = cyy + v.a[2];
    S.a[3] = cxz;
    S.a[4] = cyz;
    S.a[5] = czz + v.a[5];
    const Sym3 Si = inverse_sym3(S);
    const float r[3] = {hx - x, hy - y, hz - z};
    float c2 = 0.f;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) c2 = fmaf(r[i] * Si.a[s3(i, j)], r[j], c2);
    return c2;
}

// Kalman update with the 3x3 measurement; kJoseph selects the Joseph form of
// the covariance (the fit).  Returns the hit's chi2.
template <bool kJoseph>
__device__ __forceinline__ float kf_update_3d(float (&p)[6], float (&c)[21], Trig &tg, float hx, float hy, float hz,
                                              float var_u, float var_r, float var_z)
{
    const float irh = __builtin_amdgcn_rsqf(fmaf(hx, hx, hy * hy));
    const Sym3 v = hit_ellipsoid(hx * irh, hy * irh, var_u, var_r, var_z);
    float M[3][6];   // H C: rows 0..2 of C
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int j = 0; j < 6; ++j) M[k][j] = c[sym(k, j)];
    Sym3 S;
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        constexpr int kI[6] = {0, 0, 1, 0, 1, 2}, kJ[6] = {0, 1, 1, 2, 2, 2};
        S.a[e] = M[kI[e]][kJ[e]] + v.a[e];
    }
    const Sym3 Si = inverse_sym3(S);
    const float r[3] = {hx - p[0], hy - p[1], hz - p[2]};
    float Sr[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) Sr[i] = fmaf(Si.a[s3(i, 0)], r[0], fmaf(Si.a[s3(i, 1)], r[1], Si.a[s3(i, 2)] * r[2]));
    const float chi2 = fmaf(r[0], Sr[0], fmaf(r[1], Sr[1], r[2] * Sr[2]));
    float K[6][3];   // C H^T S^-1
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            K[i][k] = fmaf(M[0][i], Si.a[s3(0, k)], fmaf(M[1][i], Si.a[s3(1, k)], M[2][i] * Si.a[s3(2, k)]));
    float dp[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        dp[i] = fmaf(K[i][0], r[0], fmaf(K[i][1], r[1], K[i][2] * r[2]));
        p[i] += dp[i];
    }
    p[4] = wrap_pi(p[4]);
    rotate(tg.sph, tg.cph, dp[4]);
    rotate(tg.sth, tg.cth, dp[5]);
    if (!kJoseph) {
#pragma unroll
        for (int i = 0; i < 6; ++i)
#pragma unroll
            for (int j = i; j < 6; ++j)
                c[sym(i, j)] -= fmaf(K[i][0], M[0][j], fmaf(K[i][1], M[1][j], K[i][2] * M[2][j]));
        return chi2;
    }
    // C' = D - (D H^T) K^T + K V K^T with D = (I - K H) C
    float nc[21];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        float D[6];
#pragma unroll
        for (int j = 0; j < 6; ++j)
            D[j] = c[sym(i, j)] - fmaf(K[i][0], M[0][j], fmaf(K[i][1], M[1][j], K[i][2] * M[2][j]));
        float KV[3];   // row i of K V
#pragma unroll
        for (int l = 0; l < 3; ++l)
            KV[l] = fmaf(K[i][0], v.a[s3(0, l)], fmaf(K[i][1], v.a[s3(1, l)], K[i][2] * v.a[s3(2, l)]));
#pragma unroll
        for (int j = i; j < 6; ++j) {
            const float dk = fmaf(D[0], K[j][0], fmaf(D[1], K[j][1], D[2] * K[j][2]));
            const float kvk = fmaf(KV[0], K[j][0], fmaf(KV[1], K[j][1], KV[2] * K[j][2]));
            nc[sym(i, j)] = D[j] - dk + kvk;
        }
    }
#pragma unroll
    for (int i = 0; i < 21; ++i) c[i] = nc[i];
    return chi2;
}

// ---- beam ordering ---------------------------------------------------------
// A child's rank key (smaller = better; distinct within a seed), most
// significant first: 31 - n_hits (5 bits), the candidate's summed chi2 to
// 2^-15 relative (its float bits 31..8; non-negative float bits order like
// the floats), the parent's rank (3 bits), the remaining chi2 bits 7..0, the
// hit index (24 bits; kHoleId for hole and stopped entries).  Children of
// different parents whose chi2 agree to 2^-15 so rank by parent, and the
// children of one parent by exact chi2, then hit index.
__device__ __forceinline__ unsigned long long child_key(int n_hits, unsigned chi2_bits, int parent, unsigned hit)
{
    return ((unsigned long long)(31 - n_hits) << 59) | ((unsigned long long)(chi2_bits >> 8) << 35) |
           ((unsigned long long)parent << 32) | ((unsigned long long)(chi2_bits & 0xFFu) << 24) |
           (unsigned long long)(hit & kHoleId);
}
__device__ __forceinline__ int key_nhits(unsigned long long k) { return 31 - (int)(k >> 59); }
__device__ __forceinline__ float key_chi2(unsigned long long k)
{
    return __uint_as_float((((unsigned)(k >> 35) & 0xFFFFFFu) << 8) | ((unsigned)(k >> 24) & 0xFFu));
}
__device__ __forceinline__ int key_parent(unsigned long long k) { return (int)((k >> 32) & 7); }
__device__ __forceinline__ unsigned key_hit(unsigned long long k) { return (unsigned)(k & kHoleId); }

}  // namespace mkf
