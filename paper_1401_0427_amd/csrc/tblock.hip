// Two steps of the all-periodic 2D path in one launch (temporal blocking).
//
// A step of the scheme reads every population once and writes it once, so one
// launch per step is bound by 192 B (FP64) / 96 B (FP32) of HBM traffic per
// node.  Fusing two steps reads the level-n state once and writes level n+2
// once; the level-n+1 values live only in registers and LDS.
//
// Mapping: a workgroup of 512 threads owns a strip of 510 output columns
// [x0, x0 + 510) and a segment of rows [y0, y1) (24 rows by default).  Thread t computes the
// intermediate (level n+1, post-collision) node of column x0 - 1 + t, one row
// ahead of the output row it produces in the same column, marching upward.
// For its output node (x, y) the pull needs the intermediate values
//   e1 planes from (x-1, y), e3 planes from (x+1, y)  -> neighbour threads, LDS
//   e2 planes from (x, y-1), e4 planes from (x, y+1)  -> this thread's registers
// so only six planes of one row cross threads, through a double-buffered LDS
// row.  Every intermediate value is rounded to the storage type before use,
// exactly as a store and a reload would round it, and the per-node arithmetic
// (pull order, collision) is that of the one-step kernel: two fused steps give
// bit for bit the state of two single steps.  Redundant work: two halo columns
// per 510 and two halo rows per segment.  Measured at 4096^2: 512-thread strips
// and 24-row segments were fastest; segment lengths that are powers of two
// (32, 64) were 15-20 % slower with FP32 storage, prefetching the next row's
// pulls (more registers, fewer waves) slower still.
#include "internal.h"

namespace lbm {

#ifndef LBM_X2_THREADS
#define LBM_X2_THREADS 512
#endif
constexpr int kX2Threads = LBM_X2_THREADS;  // threads (columns) per workgroup
constexpr int kX2Out = kX2Threads - 2;

// Post-collision level-n+1 node (xw, yw) of the all-periodic grid, rounded to T.
template <typename T>
__device__ __forceinline__ void x2_inter(const T *__restrict__ src, const Geo &G, const Phys &P,
                                         int xm, int xw, int xp, int yw, double *f)
{
    const int nx = G.nx, ny = G.ny;
    const long ps = G.ps;
    const long row = (long)yw * nx;
    const long rm = yw == 0 ? (long)(ny - 1) * nx : row - nx;
    const long rp = yw == ny - 1 ? 0 : row + nx;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T *b = src + (4 * c) * ps;
        f[4 * c + 0] = ld(b + row + xm);
        f[4 * c + 1] = ld(b + ps + rm + xw);
        f[4 * c + 2] = ld(b + 2 * ps + row + xp);
        f[4 * c + 3] = ld(b + 3 * ps + rp + xw);
    }
    collide2d(f, P);
#pragma unroll
    for (int pl = 0; pl < 12; ++pl) f[pl] = (double)(T)f[pl];
}

template <typename T>
__global__ void __launch_bounds__(kX2Threads)
    k_step2d_x2(const T *__restrict__ src, T *__restrict__ dst, Geo G, Phys P, int nstrips,
                int seg)
{
    // e1 planes (0, 4, 8) and e3 planes (2, 6, 10) of the last two
    // intermediate rows, indexed [row parity][k][thread]
    __shared__ T lx[2][6][kX2Threads];
    const int nx = G.nx, ny = G.ny;
    const long ps = G.ps;
    const int t = threadIdx.x;
    const int strip = blockIdx.x % nstrips;
    const int x0 = strip * kX2Out;
    const int y0 = (blockIdx.x / nstrips) * seg;
    const int y1 = min(y0 + seg, ny);
    const int xo_end = min(x0 + kX2Out, nx);  // output columns [x0, xo_end)
    const int xi = x0 - 1 + t;                 // this thread's column
    const bool icol = xi <= xo_end;            // intermediate columns x0-1 .. xo_end
    const bool ocol = t >= 1 && xi < xo_end;   // output columns
    const int xw = xi < 0 ? xi + nx : (xi >= nx ? xi - nx : xi);
    const int xm = xw == 0 ? nx - 1 : xw - 1;
    const int xp = xw == nx - 1 ? 0 : xw + 1;
    auto wrapy = [ny](int y) { return y < 0 ? y + ny : (y >= ny ? y - ny : y); };

    double f[12];
    double e2m[3] = {0.0, 0.0, 0.0}, e2c[3] = {0.0, 0.0, 0.0};  // e2 planes of rows y-1, y
    if (icol) {
        x2_inter(src, G, P, xm, xw, xp, wrapy(y0 - 1), f);
        e2m[0] = f[1];
        e2m[1] = f[5];
        e2m[2] = f[9];
        x2_inter(src, G, P, xm, xw, xp, wrapy(y0), f);
        e2c[0] = f[1];
        e2c[1] = f[5];
        e2c[2] = f[9];
        const int b = y0 & 1;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            lx[b][c][t] = (T)f[4 * c];
            lx[b][3 + c][t] = (T)f[4 * c + 2];
        }
    }
    __syncthreads();
    for (int y = y0; y < y1; ++y) {
        double g[12];
        if (icol) {
            x2_inter(src, G, P, xm, xw, xp, wrapy(y + 1), g);
            const int b = (y + 1) & 1;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                lx[b][c][t] = (T)g[4 * c];
                lx[b][3 + c][t] = (T)g[4 * c + 2];
            }
        }
        if (ocol) {
            const int b = y & 1;
            double o[12];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                o[4 * c + 0] = (double)lx[b][c][t - 1];
                o[4 * c + 1] = e2m[c];
                o[4 * c + 2] = (double)lx[b][3 + c][t + 1];
                o[4 * c + 3] = g[4 * c + 3];
            }
            collide2d(o, P);
            T *out = dst + (long)y * nx + xi;
#pragma unroll
            for (int pl = 0; pl < 12; ++pl) sth<2>(out + pl * ps, o[pl]);
        }
        if (icol) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                e2m[c] = e2c[c];
                e2c[c] = g[4 * c + 1];
            }
        }
        __syncthreads();
    }
}

int step2x_blocks(const Geo &G, int seg)
{
    const int nstrips = (G.nx + kX2Out - 1) / kX2Out;
    return nstrips * ((G.ny + seg - 1) / seg);
}

hipError_t launch_step2x(bool f32, const void *src, void *dst, const Geo &G, const Phys &P,
                         int seg, hipStream_t st)
{
    const int nstrips = (G.nx + kX2Out - 1) / kX2Out;
    const int nb = step2x_blocks(G, seg);
    if (f32)
        hipLaunchKernelGGL(k_step2d_x2<float>, dim3(nb), dim3(kX2Threads), 0, st,
                           (const float *)src, (float *)dst, G, P, nstrips, seg);
    else
        hipLaunchKernelGGL(k_step2d_x2<double>, dim3(nb), dim3(kX2Threads), 0, st,
                           (const double *)src, (double *)dst, G, P, nstrips, seg);
    return hipGetLastError();
}

} // namespace lbm
