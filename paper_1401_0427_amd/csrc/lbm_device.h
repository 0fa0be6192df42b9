// Device-side building blocks of the vectorial lattice Boltzmann step
// (Dubois, Sec. 1-3, a = 0 form: D1Q2 / D2Q4 per conserved component).
//
// Arithmetic is double precision throughout; storage is double or float.
// The operation order below is fixed on purpose (pairwise sums of opposite
// directions; the library is built with -ffp-contract=off, and fused
// multiply-adds appear only where written, for float storage), so results are
// reproducible bit for bit and keep the exact reflection symmetries of the
// lattice.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

enum { BC_PERIODIC = 0, BC_NEUMANN = 1, BC_WALL = 2, BC_INFLOW = 3 };

// ---- storage ------------------------------------------------------------------
__device__ __forceinline__ double ld(const double *p) { return *p; }
__device__ __forceinline__ double ld(const float *p) { return (double)*p; }
__device__ __forceinline__ void st(double *p, double v) { *p = v; }
__device__ __forceinline__ void st(float *p, double v) { *p = (float)v; }

// Loads / stores with optional non-temporal hints (H bit 0: loads, bit 1: stores).
template <int H>
__device__ __forceinline__ double ldh(const double *p)
{
    if constexpr ((H & 1) != 0) return __builtin_nontemporal_load(p);
    else return *p;
}
template <int H>
__device__ __forceinline__ double ldh(const float *p)
{
    if constexpr ((H & 1) != 0) return (double)__builtin_nontemporal_load(p);
    else return (double)*p;
}
template <int H>
__device__ __forceinline__ void sth(double *p, double v)
{
    if constexpr ((H & 2) != 0) __builtin_nontemporal_store(v, p);
    else *p = v;
}
template <int H>
__device__ __forceinline__ void sth(float *p, double v)
{
    if constexpr ((H & 2) != 0) __builtin_nontemporal_store((float)v, p);
    else *p = (float)v;
}

// ---- physics constants of one problem -----------------------------------------
struct Phys {
    double c;   // 1 / (2 lambda)
    double s;   // relaxation rate
    double hg;  // g / 2
    double g;
};

// 1/h rounded correctly (bit for bit the IEEE quotient) for 2^-500 < h < 2^500:
// the hardware reciprocal estimate, two Newton steps, then one correction with
// the residual -- the steps of the full division sequence without its operand
// scaling and special-case fix-up, which leave such h unchanged (checked
// against the IEEE quotient on 2^32 values spread over that range, all equal).
// lbm_init rejects initial heights outside the range.
__device__ __forceinline__ double lbm_rcp(double h)
{
    double r = __builtin_amdgcn_rcp(h);
    double e = __builtin_fma(-h, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-h, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-h, r, 1.0);
    return __builtin_fma(e, r, r);
}

// a b + c for a state stored as T: double storage rounds the product and the sum
// separately (the operation order of a plain evaluation, so that results agree
// bit for bit with one); float storage fuses them, its results being rounded to
// float at every step anyway.
template <typename T>
__device__ __forceinline__ double mad(double a, double b, double c)
{
    if constexpr (sizeof(T) == 4)
        return __builtin_fma(a, b, c);
    else
        return a * b + c;
}

// Equilibria at a = 0 (closed form of the derivatives of the potentials h_j^*,
// Sec. 2 eqs. 2-potentiels-st-venant-1d(-suite) and Sec. 3 eqs.
// 3-st-venant-contraintes-2, 3-st-venant-enplus, with a = 0).
//   1D planes: f+, f-, g+, g-
//   2D planes: h e1..e4, qx e1..e4, qy e1..e4 (e1 +x, e2 +y, e3 -x, e4 -y)
// T: the storage type of the state (the arithmetic is double either way).
template <typename T>
__device__ __forceinline__ void feq1d(double h, double q, const Phys &P, double *e)
{
    const double ih = lbm_rcp(h);
    const double p = P.hg * (h * h);
    const double Fq = mad<T>(q * q, ih, p);
    const double hh = 0.5 * h, qh = 0.5 * q;
    if constexpr (sizeof(T) == 4) {
        e[0] = __builtin_fma(q, P.c, hh);
        e[1] = __builtin_fma(-q, P.c, hh);
        e[2] = __builtin_fma(Fq, P.c, qh);
        e[3] = __builtin_fma(-Fq, P.c, qh);
    } else {
        const double A = q * P.c, B = Fq * P.c;
        e[0] = hh + A;
        e[1] = hh - A;
        e[2] = qh + B;
        e[3] = qh - B;
    }
}

template <typename T>
__device__ __forceinline__ void feq2d(double h, double qx, double qy, const Phys &P, double *e)
{
    const double ih = lbm_rcp(h);
    const double p = P.hg * (h * h);
    const double Fxx = mad<T>(qx * qx, ih, p);
    const double Fxy = (qx * qy) * ih;
    const double Fyy = mad<T>(qy * qy, ih, p);
    const double hq = 0.25 * h, xq = 0.25 * qx, yq = 0.25 * qy;
    const double c = P.c;
    if constexpr (sizeof(T) == 4) {
        e[0] = __builtin_fma(qx, c, hq);   e[1] = __builtin_fma(qy, c, hq);
        e[2] = __builtin_fma(-qx, c, hq);  e[3] = __builtin_fma(-qy, c, hq);
        e[4] = __builtin_fma(Fxx, c, xq);  e[5] = __builtin_fma(Fxy, c, xq);
        e[6] = __builtin_fma(-Fxx, c, xq); e[7] = __builtin_fma(-Fxy, c, xq);
        e[8] = __builtin_fma(Fxy, c, yq);  e[9] = __builtin_fma(Fyy, c, yq);
        e[10] = __builtin_fma(-Fxy, c, yq); e[11] = __builtin_fma(-Fyy, c, yq);
    } else {
        const double A = qx * c, B = qy * c;
        const double Cxx = Fxx * c, Cxy = Fxy * c, Cyy = Fyy * c;
        e[0] = hq + A;  e[1] = hq + B;  e[2] = hq - A;  e[3] = hq - B;
        e[4] = xq + Cxx; e[5] = xq + Cxy; e[6] = xq - Cxx; e[7] = xq - Cxy;
        e[8] = yq + Cxy; e[9] = yq + Cyy; e[10] = yq - Cxy; e[11] = yq - Cyy;
    }
}

// Conserved moments W^k = sum_j f_j^k (eq. 1-hyp-N-vconserv).
__device__ __forceinline__ void moments1d(const double *f, double &h, double &q)
{
    h = f[0] + f[1];
    q = f[2] + f[3];
}

__device__ __forceinline__ void moments2d(const double *f, double &h, double &qx, double &qy)
{
    h = (f[0] + f[2]) + (f[1] + f[3]);
    qx = (f[4] + f[6]) + (f[5] + f[7]);
    qy = (f[8] + f[10]) + (f[9] + f[11]);
}

// BGK relaxation f* = f + s (f^eq(W(f)) - f) (eq. 2-relaxation, all rates equal).
template <typename T>
__device__ __forceinline__ void collide1d(double *f, const Phys &P)
{
    double h, q, e[4];
    moments1d(f, h, q);
    feq1d<T>(h, q, P, e);
#pragma unroll
    for (int i = 0; i < 4; ++i) f[i] = mad<T>(P.s, e[i] - f[i], f[i]);
}

template <typename T>
__device__ __forceinline__ void collide2d(double *f, const Phys &P)
{
    double h, qx, qy, e[12];
    moments2d(f, h, qx, qy);
    feq2d<T>(h, qx, qy, P, e);
#pragma unroll
    for (int i = 0; i < 12; ++i) f[i] = mad<T>(P.s, e[i] - f[i], f[i]);
}

// ---- XCD-aware tile order -------------------------------------------------------
// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on
// XCD b % 8).  Remapping b -> (b % 8) * (T / 8) + b / 8 gives each XCD one
// contiguous range of tiles, so the cache lines shared by neighbouring tiles
// (the x-shifted pulls) stay in one XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int ntiles, bool remap = true)
{
    if (!remap || (ntiles & 7) != 0) return b;
    return (b & 7) * (ntiles >> 3) + (b >> 3);
}

// ---- boundary pulls ----------------------------------------------------------------
// Geometry of one problem in a state buffer.
struct Geo {
    int nx, ny;
    long ps;      // plane stride (elements)
    int bc[4];    // x-, x+, y-, y+
    double win[4][3];
};

// Pull of plane `pl` (2D) at boundary node (x, y) whose upstream node is
// outside the domain through `face`.
template <typename T>
__device__ double pull_face2d(const T *__restrict__ src, const Geo &G, const Phys &P, int pl,
                              int face, int x, int y, int sx, int sy)
{
    switch (G.bc[face]) {
    case BC_PERIODIC: {
        sx = sx < 0 ? sx + G.nx : (sx >= G.nx ? sx - G.nx : sx);
        sy = sy < 0 ? sy + G.ny : (sy >= G.ny ? sy - G.ny : sy);
        return ld(src + pl * G.ps + (long)sy * G.nx + sx);
    }
    case BC_NEUMANN:
        return ld(src + pl * G.ps + (long)y * G.nx + x);
    case BC_WALL: {
        const int k = pl >> 2, j = pl & 3;
        const int opp = (k << 2) | ((j + 2) & 3);
        const int normal = face < 2 ? 1 : 2;
        const double v = ld(src + opp * G.ps + (long)y * G.nx + x);
        return k == normal ? -v : v;
    }
    default: {
        double e[12];
        feq2d<T>(G.win[face][0], G.win[face][1], G.win[face][2], P, e);
        return e[pl];
    }
    }
}

// Pull of all 12 planes at (x, y) with boundary rules wherever needed.
template <typename T>
__device__ __forceinline__ void pull2d_generic(const T *__restrict__ src, const Geo &G,
                                               const Phys &P, int x, int y, double *f)
{
    const long row = (long)y * G.nx;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const T *b = src + (4 * k) * G.ps;
        // e1 (+x): from x-1
        f[4 * k + 0] = x > 0 ? ld(b + row + x - 1)
                             : pull_face2d(src, G, P, 4 * k + 0, 0, x, y, x - 1, y);
        // e2 (+y): from y-1
        f[4 * k + 1] = y > 0 ? ld(b + G.ps + row - G.nx + x)
                             : pull_face2d(src, G, P, 4 * k + 1, 2, x, y, x, y - 1);
        // e3 (-x): from x+1
        f[4 * k + 2] = x < G.nx - 1 ? ld(b + 2 * G.ps + row + x + 1)
                                    : pull_face2d(src, G, P, 4 * k + 2, 1, x, y, x + 1, y);
        // e4 (-y): from y+1
        f[4 * k + 3] = y < G.ny - 1 ? ld(b + 3 * G.ps + row + G.nx + x)
                                    : pull_face2d(src, G, P, 4 * k + 3, 3, x, y, x, y + 1);
    }
}

// 1D: planes f+ (0), f- (1), g+ (2), g- (3); face 0 = x-, face 1 = x+.
template <typename T>
__device__ double pull_face1d(const T *__restrict__ src, const Geo &G, const Phys &P, int pl,
                              int face, int x)
{
    switch (G.bc[face]) {
    case BC_PERIODIC:
        return ld(src + pl * G.ps + (face == 0 ? G.nx - 1 : 0));
    case BC_NEUMANN:
        return ld(src + pl * G.ps + x);
    case BC_WALL: {
        const int opp = pl ^ 1;
        const double v = ld(src + opp * G.ps + x);
        return pl >= 2 ? -v : v;
    }
    default: {
        double e[4];
        feq1d<T>(G.win[face][0], G.win[face][1], P, e);
        return e[pl];
    }
    }
}

template <typename T>
__device__ __forceinline__ void pull1d(const T *__restrict__ src, const Geo &G, const Phys &P,
                                       int x, double *f)
{
    const long ps = G.ps;
    if (x > 0) {
        f[0] = ld(src + x - 1);
        f[2] = ld(src + 2 * ps + x - 1);
    } else {
        f[0] = pull_face1d(src, G, P, 0, 0, x);
        f[2] = pull_face1d(src, G, P, 2, 0, x);
    }
    if (x < G.nx - 1) {
        f[1] = ld(src + ps + x + 1);
        f[3] = ld(src + 3 * ps + x + 1);
    } else {
        f[1] = pull_face1d(src, G, P, 1, 1, x);
        f[3] = pull_face1d(src, G, P, 3, 1, x);
    }
}

} // namespace lbm
