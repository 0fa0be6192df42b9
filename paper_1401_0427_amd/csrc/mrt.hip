// The paper's schemes with a rest population: D1Q3Q2 (Sec. 2) and D2Q5Q4Q4
// (Sec. 3), rest weight a >= 0, relaxed in moment space with one rate per
// non-conserved moment (eq. 2-relaxation, MRT).
//
// Equilibria (derivatives of the potentials h_j^* with K = 1/(2g),
// theta = g h - |u|^2/2, c = 1/(2 lambda)):
//   f_0 = a K theta,
//   1D: f_+- = (h - f_0)/2 +- q c,             g_+- = q/2 +- (q u + p) c
//   2D: f_{1,3} = (h - f_0)/4 +- qx c,         f_{2,4} = (h - f_0)/4 +- qy c,
//       gx / gy as in the a = 0 scheme (the rest potential does not depend on u).
// Moments (Sec. 2, Sec. 3):
//   1D: rho = f_0 + f_+ + f_-, J = lambda (f_+ - f_-), eps = lambda^2 (f_+ + f_- - 2 f_0),
//       q = g_+ + g_-, J_q = lambda (g_+ - g_-)
//   2D: rho, J_x = lambda (f_1 - f_3), J_y = lambda (f_2 - f_4),
//       eps = f_1 + f_2 + f_3 + f_4 - 4 f_0, XX = f_1 - f_2 + f_3 - f_4;
//       per momentum family: q, lambda (g_1 - g_3), lambda (g_2 - g_4),
//       g_1 - g_2 + g_3 - g_4.
// Equilibrium moments: J^eq = q; 1D eps^eq = lambda^2 (rho - 3 a K theta),
//   J_q^eq = q u + p; 2D eps^eq = (1 - 5a/2) rho + (5a/4)(u^2 + v^2)/g (the factor a
//   of the second term restored), XX^eq = 0, f_xx^eq = rho u^2 + p,
//   f_xy^eq = f_yx^eq = rho u v, f_yy^eq = rho v^2 + p.
// Plane order: rest population first, then the a = 0 order.
#include "internal.h"
#include "xk_wave.h"
#include "multistep.h"

namespace lbm {

__device__ __forceinline__ void feq_rest1d(double h, double q, const Mrt &M, double *e)
{
    const double ih = 1.0 / h;
    const double u = q * ih;
    const double theta = M.g * h - 0.5 * (u * u);
    const double f0 = M.aK * theta;
    const double hr = h - f0;
    const double p = M.hg * (h * h);
    const double Fq = (q * q) * ih + p;
    e[0] = f0;
    e[1] = 0.5 * hr + q * M.c;
    e[2] = 0.5 * hr - q * M.c;
    e[3] = 0.5 * q + Fq * M.c;
    e[4] = 0.5 * q - Fq * M.c;
}

__device__ __forceinline__ void feq_rest2d(double h, double qx, double qy, const Mrt &M, double *e)
{
    const double ih = 1.0 / h;
    const double u = qx * ih, v = qy * ih;
    const double theta = M.g * h - 0.5 * (u * u + v * v);
    const double f0 = M.aK * theta;
    const double hr = h - f0;
    const double p = M.hg * (h * h);
    const double Fxx = (qx * qx) * ih + p, Fxy = (qx * qy) * ih, Fyy = (qy * qy) * ih + p;
    const double hq = 0.25 * hr, xq = 0.25 * qx, yq = 0.25 * qy;
    e[0] = f0;
    e[1] = hq + qx * M.c; e[2] = hq + qy * M.c; e[3] = hq - qx * M.c; e[4] = hq - qy * M.c;
    e[5] = xq + Fxx * M.c; e[6] = xq + Fxy * M.c; e[7] = xq - Fxx * M.c; e[8] = xq - Fxy * M.c;
    e[9] = yq + Fxy * M.c; e[10] = yq + Fyy * M.c; e[11] = yq - Fxy * M.c; e[12] = yq - Fyy * M.c;
}

__device__ __forceinline__ void collide_mrt1d(double *f, const Mrt &M)
{
    const double lam = M.lam, il = M.il;
    const double sp = f[1] + f[2];
    const double rho = f[0] + sp;
    double J = lam * (f[1] - f[2]);
    double eps = (lam * lam) * (sp - 2.0 * f[0]);
    const double q = f[3] + f[4];
    double Jq = lam * (f[3] - f[4]);
    const double u = q / rho;
    const double p = M.hg * (rho * rho);
    const double theta = M.g * rho - 0.5 * (u * u);
    J += M.rate[0] * (q - J);
    eps += M.rate[1] * ((lam * lam) * (rho - 3.0 * (M.aK * theta)) - eps);
    Jq += M.rate[2] * ((q * u + p) - Jq);
    const double f0 = (rho - eps * (il * il)) / 3.0;
    const double S = rho - f0;
    f[0] = f0;
    f[1] = 0.5 * (S + J * il);
    f[2] = 0.5 * (S - J * il);
    f[3] = 0.5 * (q + Jq * il);
    f[4] = 0.5 * (q - Jq * il);
}

// Moments of one momentum family (g_1..g_4): total, x- and y-moments, XX.
__device__ __forceinline__ void fam_moments(const double *g, double lam, double &q, double &mx,
                                            double &my, double &xx)
{
    const double a = g[0] + g[2], b = g[1] + g[3];
    q = a + b;
    mx = lam * (g[0] - g[2]);
    my = lam * (g[1] - g[3]);
    xx = a - b;
}

__device__ __forceinline__ void fam_invert(double *g, double il, double q, double mx, double my,
                                           double xx)
{
    const double a = 0.5 * (q + xx), b = 0.5 * (q - xx);
    g[0] = 0.5 * (a + mx * il);
    g[2] = 0.5 * (a - mx * il);
    g[1] = 0.5 * (b + my * il);
    g[3] = 0.5 * (b - my * il);
}

__device__ __forceinline__ void collide_mrt2d(double *f, const Mrt &M)
{
    const double lam = M.lam, il = M.il;
    const double *r = M.rate;
    const double s13 = f[1] + f[3], s24 = f[2] + f[4];
    const double rho = f[0] + (s13 + s24);
    double Jx = lam * (f[1] - f[3]);
    double Jy = lam * (f[2] - f[4]);
    double eps = (s13 + s24) - 4.0 * f[0];
    double XX = s13 - s24;
    double qx, fxx, fxy, XXu, qy, fyx, fyy, XXv;
    fam_moments(f + 5, lam, qx, fxx, fxy, XXu);
    fam_moments(f + 9, lam, qy, fyx, fyy, XXv);
    const double ir = 1.0 / rho;
    const double u = qx * ir, v = qy * ir;
    const double p = M.hg * (rho * rho);
    Jx += r[0] * (qx - Jx);
    Jy += r[1] * (qy - Jy);
    eps += r[2] * (((1.0 - 2.5 * M.a) * rho + (1.25 * M.a) * (u * u + v * v) / M.g) - eps);
    XX += r[3] * (0.0 - XX);
    fxx += r[4] * ((qx * u + p) - fxx);
    fxy += r[5] * (qx * v - fxy);
    XXu += r[6] * (0.0 - XXu);
    fyx += r[7] * (qy * u - fyx);
    fyy += r[8] * ((qy * v + p) - fyy);
    XXv += r[9] * (0.0 - XXv);
    const double f0 = 0.2 * (rho - eps);
    const double S = rho - f0;
    const double a = 0.5 * (S + XX), b = 0.5 * (S - XX);
    f[0] = f0;
    f[1] = 0.5 * (a + Jx * il);
    f[3] = 0.5 * (a - Jx * il);
    f[2] = 0.5 * (b + Jy * il);
    f[4] = 0.5 * (b - Jy * il);
    fam_invert(f + 5, il, qx, fxx, fxy, XXu);
    fam_invert(f + 9, il, qy, fyx, fyy, XXv);
}

// ---- pulls (rest plane 0 does not move) ---------------------------------------------
// An inflow face takes the equilibrium of its prescribed state, evaluated here in
// registers.  (Returning a value loaded from a precomputed table in the default
// case of the face switch made the compiler's control-flow structurizer drop the
// table address on one of the paths into that case, so the load went through an
// unassigned register.)
template <typename T>
__device__ double pull_rest_face2d(const T *__restrict__ src, const Geo &G, const Mrt &M, int pl,
                                   int face, int x, int y, int sx, int sy)
{
    switch (G.bc[face]) {
    case BC_PERIODIC:
        sx = sx < 0 ? sx + G.nx : (sx >= G.nx ? sx - G.nx : sx);
        sy = sy < 0 ? sy + G.ny : (sy >= G.ny ? sy - G.ny : sy);
        return ld(src + pl * G.ps + (long)sy * G.nx + sx);
    case BC_NEUMANN:
        return ld(src + pl * G.ps + (long)y * G.nx + x);
    case BC_WALL: {
        const int k = (pl - 1) >> 2, j = (pl - 1) & 3;
        const int opp = 1 + ((k << 2) | ((j + 2) & 3));
        const double v = ld(src + opp * G.ps + (long)y * G.nx + x);
        return k == (face < 2 ? 1 : 2) ? -v : v;
    }
    default: {
        double e[13];
        feq_rest2d(G.win[face][0], G.win[face][1], G.win[face][2], M, e);
        return e[pl];
    }
    }
}

template <typename T>
__device__ __forceinline__ void pull_rest2d(const T *__restrict__ src, const Geo &G, const Mrt &M,
                                            bool allper, int x, int y, double *f)
{
    const int nx = G.nx, ny = G.ny;
    const long ps = G.ps, row = (long)y * nx;
    f[0] = ld(src + row + x);
    const bool interior = x > 0 && x < nx - 1 && y > 0 && y < ny - 1;
    if (allper || interior) {
        const int xm = x == 0 ? nx - 1 : x - 1;
        const int xp = x == nx - 1 ? 0 : x + 1;
        const long rm = y == 0 ? (long)(ny - 1) * nx : row - nx;
        const long rp = y == ny - 1 ? 0 : row + nx;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const T *b = src + (1 + 4 * k) * ps;
            f[1 + 4 * k] = ld(b + row + xm);
            f[2 + 4 * k] = ld(b + ps + rm + x);
            f[3 + 4 * k] = ld(b + 2 * ps + row + xp);
            f[4 + 4 * k] = ld(b + 3 * ps + rp + x);
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int p1 = 1 + 4 * k;
        f[p1] = x > 0 ? ld(src + p1 * ps + row + x - 1)
                      : pull_rest_face2d(src, G, M, p1, 0, x, y, x - 1, y);
        f[p1 + 1] = y > 0 ? ld(src + (p1 + 1) * ps + row - nx + x)
                          : pull_rest_face2d(src, G, M, p1 + 1, 2, x, y, x, y - 1);
        f[p1 + 2] = x < nx - 1 ? ld(src + (p1 + 2) * ps + row + x + 1)
                               : pull_rest_face2d(src, G, M, p1 + 2, 1, x, y, x + 1, y);
        f[p1 + 3] = y < ny - 1 ? ld(src + (p1 + 3) * ps + row + nx + x)
                               : pull_rest_face2d(src, G, M, p1 + 3, 3, x, y, x, y + 1);
    }
}

template <typename T>
__device__ double pull_rest_face1d(const T *__restrict__ src, const Geo &G, const Mrt &M, int pl,
                                   int face, int x)
{
    switch (G.bc[face]) {
    case BC_PERIODIC:
        return ld(src + pl * G.ps + (face == 0 ? G.nx - 1 : 0));
    case BC_NEUMANN:
        return ld(src + pl * G.ps + x);
    case BC_WALL: {
        const int opp = pl == 1 ? 2 : pl == 2 ? 1 : pl == 3 ? 4 : 3;
        const double v = ld(src + opp * G.ps + x);
        return pl >= 3 ? -v : v;
    }
    default: {
        double e[5];
        feq_rest1d(G.win[face][0], G.win[face][1], M, e);
        return e[pl];
    }
    }
}

// ---- kernels -------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_step_rest2d(const T *__restrict__ src, T *__restrict__ dst,
                                                     Geo G, Mrt M, int tiles_x, int allper)
{
    const int t = blockIdx.x;
    const int y = t / tiles_x;
    const int x = (t - y * tiles_x) * 256 + threadIdx.x;
    if (x >= G.nx) return;
    double f[13];
    pull_rest2d(src, G, M, allper != 0, x, y, f);
    collide_mrt2d(f, M);
    T *o = dst + (long)y * G.nx + x;
#pragma unroll
    for (int pl = 0; pl < 13; ++pl) sth<2>(o + pl * G.ps, f[pl]);
}

template <typename T>
__global__ void __launch_bounds__(256) k_step_rest1d(const T *__restrict__ src, T *__restrict__ dst,
                                                     Geo G, Mrt M)
{
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= G.nx) return;
    const long ps = G.ps;
    double f[5];
    f[0] = ld(src + x);
    if (x > 0) {
        f[1] = ld(src + ps + x - 1);
        f[3] = ld(src + 3 * ps + x - 1);
    } else {
        f[1] = pull_rest_face1d(src, G, M, 1, 0, x);
        f[3] = pull_rest_face1d(src, G, M, 3, 0, x);
    }
    if (x < G.nx - 1) {
        f[2] = ld(src + 2 * ps + x + 1);
        f[4] = ld(src + 4 * ps + x + 1);
    } else {
        f[2] = pull_rest_face1d(src, G, M, 2, 1, x);
        f[4] = pull_rest_face1d(src, G, M, 4, 1, x);
    }
    collide_mrt1d(f, M);
#pragma unroll
    for (int pl = 0; pl < 5; ++pl) sth<2>(dst + pl * ps + x, f[pl]);
}

// ---- D2Q5Q4Q4, K steps per launch on all-periodic grids ----------------------------
// One wavefront per column strip of 64 lanes (lane l at column x0 - (K - 1) + l,
// wrapped), walking down a segment of rows.  Iteration j computes level 1 of row
// i = y0 - (K - 1) + j from the level-n pulls of that row (loaded one iteration
// ahead), then level k + 1 of row i - k from level k for k = 1 .. K - 1, so the
// levels are skewed one row apart and only level K leaves the wavefront (row
// i - (K - 1), stored when it lies in the segment).  Level k + 1 of row r pulls
// from level k: e1 / e3 of row r from lanes l - 1 / l + 1 (cross-lane, kept from
// the previous iteration), e2 of row r - 1 (kept two iterations, two arrays used
// alternately), e4 of row r + 1 (just computed), and the rest population of row r
// (kept one iteration).  Every level is rounded to the storage type, as the
// one-step kernel's store and load round it, and the collision is the same
// function, so the result equals K single steps bit for bit.  The K - 1 lanes at
// each strip edge and the first 2 (K - 1) iterations take values from outside the
// valid range and are not stored.
template <typename T>
__device__ __forceinline__ void rest2k_load(const T *__restrict__ src, long ps, int nx, int ny,
                                            int r, int xm, int xw, int xp, T (&b)[13])
{
    const long row = (long)r * nx;
    const long rm = r == 0 ? (long)(ny - 1) * nx : row - nx;
    const long rp = r == ny - 1 ? 0 : row + nx;
    b[0] = src[row + xw];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T *q = src + (1 + 4 * c) * ps;
        b[1 + 4 * c] = q[row + xm];
        b[2 + 4 * c] = q[ps + rm + xw];
        b[3 + 4 * c] = q[2 * ps + row + xp];
        b[4 + 4 * c] = q[3 * ps + rp + xw];
    }
}

template <typename T, int K>
__global__ void __launch_bounds__(256) k_step_rest2d_k(const T *__restrict__ src,
                                                       T *__restrict__ dst, Geo G, Mrt M,
                                                       int nsb, int seg)
{
    constexpr int H = K - 1, WO = 64 - 2 * H;
    const int nx = G.nx, ny = G.ny;
    const long ps = G.ps;
    const int lane = threadIdx.x & 63;
    const int strip = (blockIdx.x % nsb) * 4 + (int)(threadIdx.x >> 6);
    const int y0 = (blockIdx.x / nsb) * seg;
    if (strip * WO >= nx || y0 >= ny) return;  // whole wavefronts only
    const int y1 = y0 + seg < ny ? y0 + seg : ny;
    const int xc = strip * WO - H + lane;
    const int xw = ((xc % nx) + nx) % nx;
    const int xm = xw == 0 ? nx - 1 : xw - 1, xp = xw == nx - 1 ? 0 : xw + 1;
    const bool olane = lane >= H && lane < H + WO && xc < nx;
    T e2[2][K - 1][3], s1[K - 1][3], s3[K - 1][3], r0[K - 1];
#pragma unroll
    for (int k = 0; k < K - 1; ++k) {
        r0[k] = (T)0;
#pragma unroll
        for (int c = 0; c < 3; ++c) e2[0][k][c] = e2[1][k][c] = s1[k][c] = s3[k][c] = (T)0;
    }
    const int niter = (y1 - y0) + 2 * H;
    int rl = (((y0 - H) % ny) + ny) % ny;  // level-1 row of the last load, wrapped
    T buf[2][13];
    rest2k_load<T>(src, ps, nx, ny, rl, xm, xw, xp, buf[0]);
    for (int j = 0; j < niter; j += 2) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int orow = y0 - 2 * H + j + u;
            rl = rl == ny - 1 ? 0 : rl + 1;
            rest2k_load<T>(src, ps, nx, ny, rl, xm, xw, xp, buf[1 - u]);
            double v[13];
#pragma unroll
            for (int pl = 0; pl < 13; ++pl) v[pl] = (double)buf[u][pl];
            collide_mrt2d(v, M);  // level 1
#pragma unroll
            for (int k = 1; k < K; ++k) {
#pragma unroll
                for (int pl = 0; pl < 13; ++pl) v[pl] = (double)(T)v[pl];
                double o[13];
                o[0] = (double)r0[k - 1];
                r0[k - 1] = (T)v[0];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int b = 1 + 4 * c;
                    o[b + 0] = (double)s1[k - 1][c];
                    o[b + 1] = (double)e2[u][k - 1][c];
                    o[b + 2] = (double)s3[k - 1][c];
                    o[b + 3] = v[b + 3];
                    e2[u][k - 1][c] = (T)v[b + 1];
                    s1[k - 1][c] = xk_xch((T)v[b + 0], lane, 1);
                    s3[k - 1][c] = xk_xch((T)v[b + 2], lane, -1);
                }
                collide_mrt2d(o, M);
#pragma unroll
                for (int pl = 0; pl < 13; ++pl) v[pl] = o[pl];
            }
            if (olane && orow >= y0 && orow < y1) {
                T *q = dst + (long)orow * nx + xc;
#pragma unroll
                for (int pl = 0; pl < 13; ++pl) sth<2>(q + pl * ps, v[pl]);
            }
        }
    }
}

// ---- D1Q3Q2, K steps per launch ------------------------------------------------------
// A workgroup of kK1Threads threads holds a tile of consecutive nodes, one per thread,
// and advances it K steps with one barrier per step: the four moving planes go
// through LDS (double-buffered), the rest population stays in the thread.  The tile
// starts K nodes before its output nodes (each step invalidates one more node at
// each tile edge), or, for a domain with non-periodic ends that fits one tile
// (step1k_whole), covers the whole domain, whose ends apply the face rules, for any
// K.  Faces as in the one-step kernel: Neumann takes the node's own value of the
// plane, a wall its own opposite plane (momentum negated), an inflow face the
// equilibrium of its state; levels rounded to the storage type, so a launch equals K
// single steps bit for bit.
__device__ __forceinline__ double rest1k_face(const Geo &G, int pl, int face, const double *own,
                                              const double *weq)
{
    switch (G.bc[face]) {
    case BC_NEUMANN:
        return own[pl];
    case BC_WALL: {
        const int opp = pl == 1 ? 2 : pl == 2 ? 1 : pl == 3 ? 4 : 3;
        const double v = own[opp];
        return pl >= 3 ? -v : v;
    }
    default:  // BC_INFLOW
        return weq[face * 5 + pl];
    }
}

template <typename T>
__global__ void __launch_bounds__(kK1Threads)
    k_step_rest1d_k(const T *__restrict__ src, T *__restrict__ dst, Geo G, Mrt M, int K,
                    int nout, int whole)
{
    constexpr int NT = kK1Threads;
    __shared__ T sh[2][4][NT];
    const int t = threadIdx.x;
    const int nx = G.nx;
    const long ps = G.ps;
    const int ob = (int)blockIdx.x * nout;
    const int x0 = whole ? 0 : ob - K;
    const bool per = G.bc[0] == BC_PERIODIC;  // the two 1D faces are periodic together
    const int oe = min(ob + nout, nx);         // output nodes [ob, oe)
    const int x = x0 + t;                      // this thread's node, unwrapped
    const bool in = per || (x >= 0 && x < nx);
    const int xw = per ? ((x % nx) + nx) % nx : x;
    const int tl = t > 0 ? t - 1 : t;  // clamped neighbours (edge values are invalid anyway)
    const int tr = t < NT - 1 ? t + 1 : t;
    double weq[10];
#pragma unroll
    for (int face = 0; face < 2; ++face)
        if (G.bc[face] == BC_INFLOW) feq_rest1d(G.win[face][0], G.win[face][1], M, weq + 5 * face);
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (in) {
#pragma unroll
        for (int pl = 0; pl < 5; ++pl) v[pl] = ld(src + pl * ps + xw);
    }
#pragma unroll
    for (int pl = 1; pl < 5; ++pl) sh[0][pl - 1][t] = (T)v[pl];
    __syncthreads();
    int b = 0;
    for (int k = 0; k < K; ++k) {
        double f[5];
        f[0] = v[0];
        // f+ and g+ (planes 1, 3) from x - 1, f- and g- (planes 2, 4) from x + 1
        if (!per && x == 0) {
            f[1] = rest1k_face(G, 1, 0, v, weq);
            f[3] = rest1k_face(G, 3, 0, v, weq);
        } else {
            f[1] = (double)sh[b][0][tl];
            f[3] = (double)sh[b][2][tl];
        }
        if (!per && x == nx - 1) {
            f[2] = rest1k_face(G, 2, 1, v, weq);
            f[4] = rest1k_face(G, 4, 1, v, weq);
        } else {
            f[2] = (double)sh[b][1][tr];
            f[4] = (double)sh[b][3][tr];
        }
        collide_mrt1d(f, M);
        b ^= 1;
#pragma unroll
        for (int pl = 0; pl < 5; ++pl) v[pl] = (double)(T)f[pl];
#pragma unroll
        for (int pl = 1; pl < 5; ++pl) sh[b][pl - 1][t] = (T)v[pl];
        __syncthreads();
    }
    if (in && x >= ob && x < oe) {
#pragma unroll
        for (int pl = 0; pl < 5; ++pl) sth<2>(dst + pl * ps + xw, v[pl]);
    }
}

hipError_t launch_step_rest1k(bool f32, const void *src, void *dst, const Geo &G, const Mrt &M,
                              int K, hipStream_t st)
{
    const int whole = step1k_whole(G) ? 1 : 0;
    if (K < 1 || (!whole && 2 * K >= kK1Threads)) return hipErrorInvalidValue;
    const int nout = whole ? G.nx : kK1Threads - 2 * K;
    const int nb = whole ? 1 : (G.nx + nout - 1) / nout;
    if (f32)
        hipLaunchKernelGGL(k_step_rest1d_k<float>, dim3(nb), dim3(kK1Threads), 0, st,
                           (const float *)src, (float *)dst, G, M, K, nout, whole);
    else
        hipLaunchKernelGGL(k_step_rest1d_k<double>, dim3(nb), dim3(kK1Threads), 0, st,
                           (const double *)src, (double *)dst, G, M, K, nout, whole);
    return hipGetLastError();
}

template <typename T, int K>
static int rest2k_resident()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step_rest2d_k<T, K>, 256, 0) !=
        hipSuccess)
        return 0;
    return nb;
}

int rest2k_seg(const Geo &G, bool f32, int K, long *slots_out)
{
    int dev = 0, ncu = 0, per = 0;
    if (slots_out) *slots_out = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    switch (K) {
#define LBM_REST_OCC(KK) \
    case KK: per = f32 ? rest2k_resident<float, KK>() : rest2k_resident<double, KK>(); break;
        LBM_REST_OCC(2) LBM_REST_OCC(3) LBM_REST_OCC(4) LBM_REST_OCC(5) LBM_REST_OCC(6)
#undef LBM_REST_OCC
    default: return 0;
    }
    const long slots = (long)ncu * per;
    if (slots_out) *slots_out = slots;
    if (slots <= 0) return 0;
    const int WO = 64 - 2 * (K - 1);
    const long ngroups = ((G.nx + WO - 1) / WO + 3) / 4;
    // segment length of the fewest rows computed per wavefront over whole rounds of
    // resident workgroups (halo rows: 2 (K - 1) per segment)
    int best = 0;
    double best_cost = 0.0;
    for (int nseg = 1; nseg <= G.ny; ++nseg) {
        const int sg = (G.ny + nseg - 1) / nseg;
        if (sg < kRestMinSeg && nseg > 1) break;  // short grids: one segment
        if ((G.ny + sg - 1) / sg != nseg) continue;
        const long blocks = ngroups * nseg;
        const long rounds = (blocks + slots - 1) / slots;
        double cost = (double)rounds * (sg + 2 * (K - 1));
        if (blocks < slots) cost *= (double)slots / (double)blocks;
        if (best == 0 || cost < best_cost) {
            best = sg;
            best_cost = cost;
        }
    }
    return best;
}

long rest2k_blocks(const Geo &G, int K, int seg)
{
    const int WO = 64 - 2 * (K - 1);
    return (long)(((G.nx + WO - 1) / WO + 3) / 4) * ((G.ny + seg - 1) / seg);
}

hipError_t launch_step_rest2k(bool f32, const void *src, void *dst, const Geo &G, const Mrt &M,
                              int K, int seg, hipStream_t st)
{
    if (seg <= 0) return hipErrorInvalidValue;
    const int WO = 64 - 2 * (K - 1);
    const int nsb = ((G.nx + WO - 1) / WO + 3) / 4;
    const dim3 grid((unsigned)rest2k_blocks(G, K, seg)), block(256);
    switch (K) {
#define LBM_REST_K(KK)                                                                       \
    case KK:                                                                                 \
        if (f32)                                                                             \
            hipLaunchKernelGGL((k_step_rest2d_k<float, KK>), grid, block, 0, st,            \
                               (const float *)src, (float *)dst, G, M, nsb, seg);            \
        else                                                                                 \
            hipLaunchKernelGGL((k_step_rest2d_k<double, KK>), grid, block, 0, st,           \
                               (const double *)src, (double *)dst, G, M, nsb, seg);          \
        break;
        LBM_REST_K(2) LBM_REST_K(3) LBM_REST_K(4) LBM_REST_K(5) LBM_REST_K(6)
#undef LBM_REST_K
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// f*(0) = C(f^eq(W0)) with the same checks as the a = 0 initialisation.
template <typename T>
__global__ void __launch_bounds__(256) k_init_rest(int dim, T *__restrict__ dst,
                                                   const double *__restrict__ h0,
                                                   const double *__restrict__ qx0,
                                                   const double *__restrict__ qy0, Geo G, Mrt M,
                                                   unsigned long long *speed_bits, int *bad)
{
    const long n = (long)G.nx * G.ny;
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double h = h0[i];
    const double qx = qx0 ? qx0[i] : 0.0;
    const double qy = (dim == 2 && qy0) ? qy0[i] : 0.0;
    if (!(h > 0.0) || !isfinite(h) || !isfinite(qx) || !isfinite(qy)) {
        atomicOr(bad, 1);
        return;
    }
    const double u = fabs(qx / h), v = fabs(qy / h);
    const double spd = (u > v ? u : v) + sqrt(M.g * h);
    atomicMax(speed_bits, (unsigned long long)__double_as_longlong(spd));
    if (dim == 1) {
        double f[5];
        feq_rest1d(h, qx, M, f);
        collide_mrt1d(f, M);
#pragma unroll
        for (int pl = 0; pl < 5; ++pl) st(dst + pl * G.ps + i, f[pl]);
    } else {
        double f[13];
        feq_rest2d(h, qx, qy, M, f);
        collide_mrt2d(f, M);
#pragma unroll
        for (int pl = 0; pl < 13; ++pl) st(dst + pl * G.ps + i, f[pl]);
    }
}

// Conserved fields, per-block partial sums (fixed order) and the divergence flag.
template <typename T>
__global__ void __launch_bounds__(256) k_moments_rest(int dim, const T *__restrict__ state,
                                                      double *__restrict__ h,
                                                      double *__restrict__ qx,
                                                      double *__restrict__ qy,
                                                      double *__restrict__ partials, int *flag,
                                                      Geo G)
{
    __shared__ double sh[3][256];
    const long n = (long)G.nx * G.ny;
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    double w[3] = {0.0, 0.0, 0.0};
    if (i < n) {
        const long ps = G.ps;
        if (dim == 1) {
            w[0] = ld(state + i) + (ld(state + ps + i) + ld(state + 2 * ps + i));
            w[1] = ld(state + 3 * ps + i) + ld(state + 4 * ps + i);
        } else {
            double f[13];
#pragma unroll
            for (int pl = 0; pl < 13; ++pl) f[pl] = ld(state + pl * ps + i);
            w[0] = f[0] + ((f[1] + f[3]) + (f[2] + f[4]));
            w[1] = (f[5] + f[7]) + (f[6] + f[8]);
            w[2] = (f[9] + f[11]) + (f[10] + f[12]);
        }
        if (h) h[i] = w[0];
        if (qx) qx[i] = w[1];
        if (qy && dim == 2) qy[i] = w[2];
        if (flag && (!(w[0] > 0.0) || !isfinite(w[0]) || !isfinite(w[1]) || !isfinite(w[2])))
            atomicOr(flag, 1);
    }
    if (partials) {
        const int t = threadIdx.x;
        for (int c = 0; c < 3; ++c) sh[c][t] = w[c];
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (t < s)
                for (int c = 0; c < 3; ++c) sh[c][t] = sh[c][t] + sh[c][t + s];
            __syncthreads();
        }
        if (t == 0)
            for (int c = 0; c < 3; ++c) partials[(long)blockIdx.x * 3 + c] = sh[c][0];
    }
}

// ---- launchers -----------------------------------------------------------------------------
hipError_t launch_init_rest(int dim, bool f32, void *dst, const double *h0, const double *qx0,
                            const double *qy0, const Geo &G, const Mrt &M,
                            unsigned long long *speed_bits, int *bad, hipStream_t st)
{
    const int nb = (int)(((long)G.nx * G.ny + 255) / 256);
    if (f32)
        hipLaunchKernelGGL(k_init_rest<float>, dim3(nb), dim3(256), 0, st, dim, (float *)dst, h0,
                           qx0, qy0, G, M, speed_bits, bad);
    else
        hipLaunchKernelGGL(k_init_rest<double>, dim3(nb), dim3(256), 0, st, dim, (double *)dst,
                           h0, qx0, qy0, G, M, speed_bits, bad);
    return hipGetLastError();
}

hipError_t launch_step_rest(int dim, bool f32, const void *src, void *dst, const Geo &G,
                            const Mrt &M, hipStream_t st)
{
    if (dim == 2) {
        const int tiles_x = (G.nx + 255) / 256;
        const int allper = G.bc[0] == BC_PERIODIC && G.bc[1] == BC_PERIODIC &&
                           G.bc[2] == BC_PERIODIC && G.bc[3] == BC_PERIODIC;
        if (f32)
            hipLaunchKernelGGL(k_step_rest2d<float>, dim3(tiles_x * G.ny), dim3(256), 0, st,
                               (const float *)src, (float *)dst, G, M, tiles_x, allper);
        else
            hipLaunchKernelGGL(k_step_rest2d<double>, dim3(tiles_x * G.ny), dim3(256), 0, st,
                               (const double *)src, (double *)dst, G, M, tiles_x, allper);
    } else {
        const int nb = (G.nx + 255) / 256;
        if (f32)
            hipLaunchKernelGGL(k_step_rest1d<float>, dim3(nb), dim3(256), 0, st,
                               (const float *)src, (float *)dst, G, M);
        else
            hipLaunchKernelGGL(k_step_rest1d<double>, dim3(nb), dim3(256), 0, st,
                               (const double *)src, (double *)dst, G, M);
    }
    return hipGetLastError();
}

hipError_t launch_moments_rest(int dim, bool f32, const void *state, double *h, double *qx,
                               double *qy, double *partials, int *flag, const Geo &G,
                               hipStream_t st, int *nblocks_out)
{
    const int nb = (int)(((long)G.nx * G.ny + 255) / 256);
    if (nblocks_out) *nblocks_out = nb;
    if (f32)
        hipLaunchKernelGGL(k_moments_rest<float>, dim3(nb), dim3(256), 0, st, dim,
                           (const float *)state, h, qx, qy, partials, flag, G);
    else
        hipLaunchKernelGGL(k_moments_rest<double>, dim3(nb), dim3(256), 0, st, dim,
                           (const double *)state, h, qx, qy, partials, flag, G);
    return hipGetLastError();
}

} // namespace lbm
