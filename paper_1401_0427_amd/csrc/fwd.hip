// Forward kernels of the vectorial lattice Boltzmann step on gfx950:
// fused pull-stream + BGK collision (one kernel per time step), level-0
// initialisation, conserved moments with deterministic FP64 totals, and the
// divergence check.
//
// Memory layout: SoA planes (one per component and direction), row-major
// [y][x]; a wavefront covers 64 consecutive x of one row so every plane access
// is a contiguous 512 B (FP64) / 256 B (FP32) segment.  The x-shifted pulls
// (e1, e3) straddle one extra cache line that the neighbouring wavefront of the
// same workgroup (or the next workgroup on the same XCD) also reads, so each
// population is still fetched from HBM once per step.
#include "internal.h"

namespace lbm {

// ------------------------------------------------------------------ 2D step ----
template <typename T, bool ALLPER, int NPT, int H>
__global__ void __launch_bounds__(512) k_step2d(const T *__restrict__ src, T *__restrict__ dst,
                                                Geo G, Phys P, int tiles_x, int ntiles,
                                                int remap)
{
    const int t = xcd_tile(blockIdx.x, ntiles, remap != 0);
    const int y = t / tiles_x;
    const int tx = t - y * tiles_x;
    const int xb = tx * (int)(blockDim.x * NPT) + threadIdx.x;
    const long ps = G.ps;
    const int nx = G.nx, ny = G.ny;
    const long row = (long)y * nx;
    double f[NPT][12];

#pragma unroll
    for (int i = 0; i < NPT; ++i) {
        const int x = xb + i * (int)blockDim.x;
        if (x >= nx) continue;
        const bool interior = x > 0 && x < nx - 1 && y > 0 && y < ny - 1;
        if (ALLPER || interior) {
            const int xm = x == 0 ? nx - 1 : x - 1;
            const int xp = x == nx - 1 ? 0 : x + 1;
            const long rm = (y == 0 ? (long)(ny - 1) * nx : row - nx);
            const long rp = (y == ny - 1 ? 0 : row + nx);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const T *b = src + (4 * k) * ps;
                f[i][4 * k + 0] = ldh<H>(b + row + xm);
                f[i][4 * k + 1] = ldh<H>(b + ps + rm + x);
                f[i][4 * k + 2] = ldh<H>(b + 2 * ps + row + xp);
                f[i][4 * k + 3] = ldh<H>(b + 3 * ps + rp + x);
            }
        } else {
            pull2d_generic(src, G, P, x, y, f[i]);
        }
    }
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
        const int x = xb + i * (int)blockDim.x;
        if (x >= nx) continue;
        collide2d<T>(f[i], P);
        T *o = dst + row + x;
#pragma unroll
        for (int pl = 0; pl < 12; ++pl) sth<H>(o + pl * ps, f[i][pl]);
    }
}

// ------------------------------------------------------------------ 1D step ----
template <typename T, int NPT, int H>
__global__ void __launch_bounds__(512) k_step1d(const T *__restrict__ src, T *__restrict__ dst,
                                                Geo G, Phys P, int ntiles, int remap)
{
    const int t = xcd_tile(blockIdx.x, ntiles, remap != 0);
    const int xb = t * (int)(blockDim.x * NPT) + threadIdx.x;
    const long ps = G.ps;
    double f[NPT][4];
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
        const int x = xb + i * (int)blockDim.x;
        if (x >= G.nx) continue;
        pull1d(src, G, P, x, f[i]);
    }
#pragma unroll
    for (int i = 0; i < NPT; ++i) {
        const int x = xb + i * (int)blockDim.x;
        if (x >= G.nx) continue;
        collide1d<T>(f[i], P);
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) sth<H>(dst + pl * ps + x, f[i][pl]);
    }
}

// ------------------------------------------------------------- initial state ----
// f*(0) = C(f^eq(W0)); also records max(|u| + sqrt(g h)) (as the bit pattern of
// a non-negative double, whose integer order is the numeric order) and flags
// h <= 0 or non-finite input.
template <typename T>
__global__ void __launch_bounds__(256) k_init(int dim, T *__restrict__ dst,
                                              const double *__restrict__ h0,
                                              const double *__restrict__ qx0,
                                              const double *__restrict__ qy0, Geo G, Phys P,
                                              unsigned long long *speed_bits, int *bad)
{
    const long n = (long)G.nx * G.ny;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double h = h0[i];
    const double qx = qx0 ? qx0[i] : 0.0;
    const double qy = (dim == 2 && qy0) ? qy0[i] : 0.0;
    // heights in (2^-500, 2^500): the range in which lbm_rcp is the IEEE quotient
    if (!(h > 0x1p-500 && h < 0x1p500) || !isfinite(qx) || !isfinite(qy)) {
        atomicOr(bad, 1);
        return;
    }
    const double u = fabs(qx / h), v = fabs(qy / h);
    const double spd = (u > v ? u : v) + sqrt(P.g * h);
    atomicMax(speed_bits, (unsigned long long)__double_as_longlong(spd));
    if (dim == 1) {
        double f[4];
        feq1d<T>(h, qx, P, f);
        collide1d<T>(f, P);
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) st(dst + pl * G.ps + i, f[pl]);
    } else {
        double f[12];
        feq2d<T>(h, qx, qy, P, f);
        collide2d<T>(f, P);
#pragma unroll
        for (int pl = 0; pl < 12; ++pl) st(dst + pl * G.ps + i, f[pl]);
    }
}

// ---------------------------------------------------------- block reduction ----
// Fixed-order tree in LDS: the result depends only on the inputs, not on timing.
template <int NC>
__device__ __forceinline__ void block_sum(double (*sh)[256], double *v)
{
    const int t = threadIdx.x;
#pragma unroll
    for (int c = 0; c < NC; ++c) sh[c][t] = v[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
#pragma unroll
            for (int c = 0; c < NC; ++c) sh[c][t] = sh[c][t] + sh[c][t + w];
        }
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = sh[c][0];
}

// ------------------------------------------------------------------- moments ----
template <typename T>
__global__ void __launch_bounds__(256) k_moments(int dim, const T *__restrict__ state,
                                                 double *__restrict__ h, double *__restrict__ qx,
                                                 double *__restrict__ qy,
                                                 double *__restrict__ partials, Geo G)
{
    __shared__ double sh[3][256];
    const long n = (long)G.nx * G.ny;
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    double w[3] = {0.0, 0.0, 0.0};
    if (i < n) {
        if (dim == 1) {
            double f[4];
#pragma unroll
            for (int pl = 0; pl < 4; ++pl) f[pl] = ld(state + pl * G.ps + i);
            moments1d(f, w[0], w[1]);
        } else {
            double f[12];
#pragma unroll
            for (int pl = 0; pl < 12; ++pl) f[pl] = ld(state + pl * G.ps + i);
            moments2d(f, w[0], w[1], w[2]);
        }
        if (h) h[i] = w[0];
        if (qx) qx[i] = w[1];
        if (qy && dim == 2) qy[i] = w[2];
    }
    if (partials) {
        block_sum<3>(sh, w);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) partials[(long)blockIdx.x * 3 + c] = w[c];
        }
    }
}

// out[c] = sum_j in[j * stride + c], one workgroup per component, fixed order.
__global__ void __launch_bounds__(256) k_sum(const double *__restrict__ in, long n, int stride,
                                             double *__restrict__ out)
{
    __shared__ double sh[1][256];
    const int c = blockIdx.x;
    double acc = 0.0;
    for (long j = threadIdx.x; j < n; j += 256) acc += in[j * stride + c];
    double v[1] = {acc};
    block_sum<1>(sh, v);
    if (threadIdx.x == 0) out[c] = v[0];
}

// ------------------------------------------------------------------- check ----
template <typename T>
__global__ void __launch_bounds__(256) k_check(int dim, const T *__restrict__ state, Geo G,
                                               int *flag)
{
    const long n = (long)G.nx * G.ny;
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double h, qx, qy = 0.0;
    if (dim == 1) {
        double f[4];
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) f[pl] = ld(state + pl * G.ps + i);
        moments1d(f, h, qx);
    } else {
        double f[12];
#pragma unroll
        for (int pl = 0; pl < 12; ++pl) f[pl] = ld(state + pl * G.ps + i);
        moments2d(f, h, qx, qy);
    }
    if (!(h > 0.0) || !isfinite(h) || !isfinite(qx) || !isfinite(qy)) atomicOr(flag, 1);
}

// ----------------------------------------------------------------- launchers ----
static inline int blocks_for(long n, int b) { return (int)((n + b - 1) / b); }

int moments_blocks(const Geo &G) { return blocks_for((long)G.nx * G.ny, 256); }

hipError_t launch_init(int dim, bool f32, void *dst, const double *h0, const double *qx0,
                       const double *qy0, const Geo &G, const Phys &P, const Launch &,
                       unsigned long long *speed_bits, int *bad, hipStream_t st)
{
    const int nb = blocks_for((long)G.nx * G.ny, 256);
    if (f32)
        hipLaunchKernelGGL(k_init<float>, dim3(nb), dim3(256), 0, st, dim, (float *)dst, h0, qx0,
                           qy0, G, P, speed_bits, bad);
    else
        hipLaunchKernelGGL(k_init<double>, dim3(nb), dim3(256), 0, st, dim, (double *)dst, h0,
                           qx0, qy0, G, P, speed_bits, bad);
    return hipGetLastError();
}

template <typename T, int NPT, int H>
static void step2d_h(bool allper, const void *src, void *dst, const Geo &G, const Phys &P,
                     const Launch &L, hipStream_t st)
{
    const int span = L.block * NPT;
    const int tiles_x = (G.nx + span - 1) / span;
    const int ntiles = tiles_x * G.ny;
    const int remap = (L.hints & 4) ? 0 : 1;
    if (allper)
        hipLaunchKernelGGL((k_step2d<T, true, NPT, H>), dim3(ntiles), dim3(L.block), 0, st,
                           (const T *)src, (T *)dst, G, P, tiles_x, ntiles, remap);
    else
        hipLaunchKernelGGL((k_step2d<T, false, NPT, 0>), dim3(ntiles), dim3(L.block), 0, st,
                           (const T *)src, (T *)dst, G, P, tiles_x, ntiles, remap);
}

template <typename T, int NPT, int H>
static void step1d_h(const void *src, void *dst, const Geo &G, const Phys &P, const Launch &L,
                     hipStream_t st)
{
    const int span = L.block * NPT;
    const int ntiles = (G.nx + span - 1) / span;
    const int remap = (L.hints & 4) ? 0 : 1;
    hipLaunchKernelGGL((k_step1d<T, NPT, H>), dim3(ntiles), dim3(L.block), 0, st,
                       (const T *)src, (T *)dst, G, P, ntiles, remap);
}

template <typename T, int NPT>
static void step_npt(int dim, bool allper, const void *src, void *dst, const Geo &G,
                     const Phys &P, const Launch &L, hipStream_t st)
{
    switch (L.hints & 3) {
    case 1:
        dim == 2 ? step2d_h<T, NPT, 1>(allper, src, dst, G, P, L, st)
                 : step1d_h<T, NPT, 1>(src, dst, G, P, L, st);
        break;
    case 2:
        dim == 2 ? step2d_h<T, NPT, 2>(allper, src, dst, G, P, L, st)
                 : step1d_h<T, NPT, 2>(src, dst, G, P, L, st);
        break;
    case 3:
        dim == 2 ? step2d_h<T, NPT, 3>(allper, src, dst, G, P, L, st)
                 : step1d_h<T, NPT, 3>(src, dst, G, P, L, st);
        break;
    default:
        dim == 2 ? step2d_h<T, NPT, 0>(allper, src, dst, G, P, L, st)
                 : step1d_h<T, NPT, 0>(src, dst, G, P, L, st);
        break;
    }
}

template <typename T>
static void step_t(int dim, const void *src, void *dst, const Geo &G, const Phys &P,
                   const Launch &L, hipStream_t st)
{
    const bool allper = G.bc[0] == BC_PERIODIC && G.bc[1] == BC_PERIODIC &&
                        G.bc[2] == BC_PERIODIC && G.bc[3] == BC_PERIODIC;
    switch (L.npt) {
    case 2: step_npt<T, 2>(dim, allper, src, dst, G, P, L, st); break;
    case 4: step_npt<T, 4>(dim, allper, src, dst, G, P, L, st); break;
    default: step_npt<T, 1>(dim, allper, src, dst, G, P, L, st); break;
    }
}

hipError_t launch_step(int dim, bool f32, const void *src, void *dst, const Geo &G,
                       const Phys &P, const Launch &L, hipStream_t st)
{
    if (f32)
        step_t<float>(dim, src, dst, G, P, L, st);
    else
        step_t<double>(dim, src, dst, G, P, L, st);
    return hipGetLastError();
}

hipError_t launch_moments(int dim, bool f32, const void *state, double *h, double *qx,
                          double *qy, double *partials, const Geo &G, hipStream_t st,
                          int *nblocks_out)
{
    const int nb = moments_blocks(G);
    if (nblocks_out) *nblocks_out = nb;
    if (f32)
        hipLaunchKernelGGL(k_moments<float>, dim3(nb), dim3(256), 0, st, dim,
                           (const float *)state, h, qx, qy, partials, G);
    else
        hipLaunchKernelGGL(k_moments<double>, dim3(nb), dim3(256), 0, st, dim,
                           (const double *)state, h, qx, qy, partials, G);
    return hipGetLastError();
}

hipError_t launch_sum(const double *in, long n, int stride, int ncomp, double *out,
                      hipStream_t st)
{
    hipLaunchKernelGGL(k_sum, dim3(ncomp), dim3(256), 0, st, in, n, stride, out);
    return hipGetLastError();
}

hipError_t launch_check(int dim, bool f32, const void *state, const Geo &G, int *flag,
                        hipStream_t st)
{
    const int nb = moments_blocks(G);
    if (f32)
        hipLaunchKernelGGL(k_check<float>, dim3(nb), dim3(256), 0, st, dim,
                           (const float *)state, G, flag);
    else
        hipLaunchKernelGGL(k_check<double>, dim3(nb), dim3(256), 0, st, dim,
                           (const double *)state, G, flag);
    return hipGetLastError();
}

} // namespace lbm
