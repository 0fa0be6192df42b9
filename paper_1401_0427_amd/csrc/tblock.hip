// Several steps per launch (temporal blocking): two steps of the all-periodic
// 2D path, and K steps of the 1D path.
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
#include <type_traits>

#include "internal.h"
#include "xk_wave.h"

namespace lbm {

constexpr int kX2Threads = 512;  // threads (columns) per workgroup
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
    collide2d<T>(f, P);
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
            collide2d<T>(o, P);
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

template <typename T, int K, int D>
__global__ void __launch_bounds__(64 * kXkWaves)
    k_step2d_xk(const T *__restrict__ src, T *__restrict__ dst, Geo G, Phys P, int nstrips,
                int seg)
{
    const int nseg = (G.ny + seg - 1) / seg;
    if constexpr (xk_sw<T>() > 1) {
        // one strip per workgroup; every wavefront runs to the end (barriers)
        constexpr int SW = xk_sw<T>();
        constexpr int rows = xk_wide_rows<T, K, SW>();
        __shared__ T lds[kXkWaves * rows];
        const int tile = xk_tile(blockIdx.x, nstrips * nseg, true);
        const int strip = tile % nstrips;
        const int y0 = (tile / nstrips) * seg;
        xk_wave<T, K, D, false, SW, true>(src, dst, G, P, strip, y0, min(y0 + seg, G.ny), lds,
                                          rows);
    } else {
        __shared__ T xs[kXkWaves][xk_lds_elems<T, K>()];
        const int ngroups = (nstrips + kXkWaves - 1) / kXkWaves;
        const int tile = xk_tile(blockIdx.x, ngroups * nseg, true);
        const int strip = (tile % ngroups) * kXkWaves + (threadIdx.x >> 6);
        if (strip >= nstrips) return;  // whole wavefront; nothing here waits on others
        const int y0 = (tile / ngroups) * seg;
        xk_wave<T, K, D, false, 1, true>(src, dst, G, P, strip, y0, min(y0 + seg, G.ny),
                                         xs[threadIdx.x >> 6]);
    }
}

// Grids with non-periodic faces (the one-step kernel's face rules); K at most
// kXkMaxKBnd.
template <typename T, int K, int D>
__global__ void __launch_bounds__(64 * kXkWaves)
    k_step2d_xkb(const T *__restrict__ src, T *__restrict__ dst, Geo G, Phys P, int nstrips,
                 int seg)
{
    __shared__ __align__(16) T xs[kXkWaves][xkb_lds_elems<T, K>()];
    const int ngroups = (nstrips + kXkWaves - 1) / kXkWaves;
    const int nseg = (G.ny + seg - 1) / seg;
    const int tile = xk_tile(blockIdx.x, ngroups * nseg, true);
    const int strip = (tile % ngroups) * kXkWaves + (threadIdx.x >> 6);
    if (strip >= nstrips) return;  // whole wavefront; nothing here waits on others
    const int y0 = (tile / ngroups) * seg;
    xk_wave<T, K, D, true, 1, true>(src, dst, G, P, strip, y0, min(y0 + seg, G.ny),
                                    xs[threadIdx.x >> 6]);
}

// Batched form: workgroup b takes tile b' (the XCD-contiguous order of b) of a
// tile table spanning many all-periodic 2D instances packed in one buffer.  A
// tile is one wide strip (xk_batch_sw > 1) or kXkWaves 64-lane strips.
template <typename T, int K, int D>
__global__ void __launch_bounds__(64 * kXkWaves)
    k_batch_xk(const InstDev *__restrict__ inst, const XkTileDev *__restrict__ tiles, int ntiles,
               const T *__restrict__ src, T *__restrict__ dst)
{
    const XkTileDev td = tiles[xk_tile(blockIdx.x, ntiles, true)];
    const InstDev &I = inst[td.inst];
    if constexpr (xk_batch_sw<T>() > 1) {
        // every wavefront runs to the end (barriers)
        constexpr int SW = xk_batch_sw<T>();
        constexpr int rows = xk_wide_rows<T, K, SW>();
        __shared__ T lds[kXkWaves * rows];
        xk_wave<T, K, D, false, SW>(src + I.off, dst + I.off, I.G, I.P, td.strip0, td.y0, td.y1,
                                    lds, rows);
    } else {
        __shared__ T xs[kXkWaves][xk_lds_elems<T, K>()];
        const int strip = td.strip0 + (int)(threadIdx.x >> 6);
        if (strip >= td.nstrips) return;
        xk_wave<T, K, D>(src + I.off, dst + I.off, I.G, I.P, strip, td.y0, td.y1,
                         xs[threadIdx.x >> 6]);
    }
}

// Output columns per strip: bnd -- the bounded kernel; else the all-periodic
// kernel with sw wavefronts per strip (1, or xk_sw of the storage type).
// Batched form, 2D instances with non-periodic faces (the bounded kernel; tiles
// of its strip geometry, K at most kXkMaxKBnd).
template <typename T, int K, int D>
__global__ void __launch_bounds__(64 * kXkWaves)
    k_batch_xkb(const InstDev *__restrict__ inst, const XkTileDev *__restrict__ tiles,
                int ntiles, const T *__restrict__ src, T *__restrict__ dst)
{
    __shared__ __align__(16) T xs[kXkWaves][xkb_lds_elems<T, K>()];
    const XkTileDev td = tiles[xk_tile(blockIdx.x, ntiles, true)];
    const InstDev &I = inst[td.inst];
    const int strip = td.strip0 + (int)(threadIdx.x >> 6);
    if (strip >= td.nstrips) return;
    xk_wave<T, K, D, true>(src + I.off, dst + I.off, I.G, I.P, strip, td.y0, td.y1,
                           xs[threadIdx.x >> 6]);
}

static int xk_wo_of(bool f32, int K, bool bnd = false, int sw = 1)
{
    if (sw > 1 && !bnd) switch (K) {
        case 2: return f32 ? xk_wo<float, 2, false, xk_sw<float>()>()
                       : xk_wo<double, 2, false, xk_sw<double>()>();
        case 3: return f32 ? xk_wo<float, 3, false, xk_sw<float>()>()
                       : xk_wo<double, 3, false, xk_sw<double>()>();
        case 4: return f32 ? xk_wo<float, 4, false, xk_sw<float>()>()
                       : xk_wo<double, 4, false, xk_sw<double>()>();
        case 5: return f32 ? xk_wo<float, 5, false, xk_sw<float>()>()
                       : xk_wo<double, 5, false, xk_sw<double>()>();
        case 6: return f32 ? xk_wo<float, 6, false, xk_sw<float>()>()
                       : xk_wo<double, 6, false, xk_sw<double>()>();
        case 7: return f32 ? xk_wo<float, 7, false, xk_sw<float>()>()
                       : xk_wo<double, 7, false, xk_sw<double>()>();
        default: return f32 ? xk_wo<float, 8, false, xk_sw<float>()>()
                       : xk_wo<double, 8, false, xk_sw<double>()>();
        }
    if (bnd) switch (K) {
        case 2: return f32 ? xk_wo<float, 2, true>() : xk_wo<double, 2, true>();
        case 3: return f32 ? xk_wo<float, 3, true>() : xk_wo<double, 3, true>();
        case 4: return f32 ? xk_wo<float, 4, true>() : xk_wo<double, 4, true>();
        case 5: return f32 ? xk_wo<float, 5, true>() : xk_wo<double, 5, true>();
        case 6: return f32 ? xk_wo<float, 6, true>() : xk_wo<double, 6, true>();
        case 7: return f32 ? xk_wo<float, 7, true>() : xk_wo<double, 7, true>();
        default: return f32 ? xk_wo<float, 8, true>() : xk_wo<double, 8, true>();
        }
    switch (K) {
    case 2: return f32 ? xk_wo<float, 2>() : xk_wo<double, 2>();
    case 3: return f32 ? xk_wo<float, 3>() : xk_wo<double, 3>();
    case 4: return f32 ? xk_wo<float, 4>() : xk_wo<double, 4>();
    case 5: return f32 ? xk_wo<float, 5>() : xk_wo<double, 5>();
    case 6: return f32 ? xk_wo<float, 6>() : xk_wo<double, 6>();
    case 7: return f32 ? xk_wo<float, 7>() : xk_wo<double, 7>();
    default: return f32 ? xk_wo<float, 8>() : xk_wo<double, 8>();
    }
}

static bool geo_bounded(const Geo &G)
{
    return G.bc[0] != BC_PERIODIC || G.bc[1] != BC_PERIODIC || G.bc[2] != BC_PERIODIC ||
           G.bc[3] != BC_PERIODIC;
}

static int step2k_strips(const Geo &G, bool f32, int K)
{
    const bool bnd = geo_bounded(G);
    const int sw = f32 ? xk_sw<float>() : xk_sw<double>();
    const int wo = xk_wo_of(f32, K, bnd, bnd ? 1 : sw);
    return (G.nx + wo - 1) / wo;
}

// Workgroups across the grid: one per wide strip, else one per kXkWaves strips.
static int step2k_groups(const Geo &G, bool f32, int K)
{
    const int ns = step2k_strips(G, f32, K);
    const int sw = f32 ? xk_sw<float>() : xk_sw<double>();
    return sw > 1 && !geo_bounded(G) ? ns : (ns + kXkWaves - 1) / kXkWaves;
}

int step2k_blocks(const Geo &G, bool f32, int K, int seg)
{
    const int ngroups = step2k_groups(G, f32, K);
    return ngroups * ((G.ny + seg - 1) / seg);
}


int step2k_max_k_bounded() { return kXkMaxKBnd; }
int step2k_default_k_bounded(bool f32)
{
    const int k = f32 ? kXkbDefaultKF32 : kXkbDefaultKF64;
    return k < kXkMaxKBnd ? k : kXkMaxKBnd;
}

template <typename T, int KK>
static hipError_t xkb_occupancy(int *n, int bs)
{
    if constexpr (KK <= kXkMaxKBnd)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(n, k_step2d_xkb<T, KK, kXkbDepth>,
                                                            bs, 0);
    else
        return hipErrorInvalidValue;
}

template <typename T, int KK>
static hipError_t xkb_launch(dim3 grid, dim3 block, hipStream_t st, const T *src, T *dst,
                             const Geo &G, const Phys &P, int ns, int seg)
{
    if constexpr (KK <= kXkMaxKBnd) {
        hipLaunchKernelGGL((k_step2d_xkb<T, KK, kXkbDepth>), grid, block, 0, st, src, dst, G, P,
                           ns, seg);
        return hipSuccess;
    } else {
        return hipErrorInvalidValue;
    }
}

// Workgroups of the K-step launch resident per compute unit (occupancy API);
// bnd: the kernel for grids with non-periodic faces.
static int xk_per_cu(bool f32, int K, bool bnd)
{
    int n = 0;
    const int bs = 64 * kXkWaves;
    hipError_t e = hipErrorInvalidValue;
#define LBM_XK_OCC(KK)                                                                        \
    case KK:                                                                                  \
        if (bnd)                                                                              \
            e = f32 ? xkb_occupancy<float, KK>(&n, bs) : xkb_occupancy<double, KK>(&n, bs);   \
        else                                                                                  \
            e = f32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(                           \
                          &n, k_step2d_xk<float, KK, kXkDepth>, bs, 0)                        \
                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(                           \
                          &n, k_step2d_xk<double, KK, kXkDepth>, bs, 0);                      \
        break;
    switch (K) {
        LBM_XK_OCC(2)
        LBM_XK_OCC(3)
        LBM_XK_OCC(4)
        LBM_XK_OCC(5)
        LBM_XK_OCC(6)
        LBM_XK_OCC(7)
        LBM_XK_OCC(8)
    default:
        break;
    }
#undef LBM_XK_OCC
    return e == hipSuccess ? n : 0;
}

// Rows per segment of the K-step launch.  Every wavefront of the launch runs
// seg + 2 (K - 1) row iterations and the workgroups run in rounds of `slots`
// (resident workgroups on the whole device), so the launch takes about
//     ceil(blocks / slots) * (seg + 2 (K - 1))
// iteration times (a partly filled single round proportionally longer: fewer
// wavefronts share the memory system).  Return the seg >= min_seg that minimises
// this, in *full whether that choice fills at least a third of the device (below
// that the few wavefronts cannot keep the memory system busy: a 512^2 FP32 grid
// at 12 % ran slower than one step per launch, FP64 at 37 % faster) and in
// *slots_out the resident workgroups; 0 when the device cannot be queried.
int step2k_seg(const Geo &G, bool f32, int K, int min_seg, bool *full, long *slots_out)
{
    int dev = 0, ncu = 0;
    if (full) *full = false;
    if (slots_out) *slots_out = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    const long slots = (long)ncu * xk_per_cu(f32, K, geo_bounded(G));
    if (slots_out) *slots_out = slots;
    if (slots <= 0) return 0;
    const long ngroups = step2k_groups(G, f32, K);
    int best = 0;
    double best_cost = 0.0;
    bool best_full = false;
    for (int nseg = 1; nseg <= G.ny; ++nseg) {
        const int seg = (G.ny + nseg - 1) / nseg;
        if (seg < min_seg) break;
        if ((G.ny + seg - 1) / seg != nseg) continue;  // same seg as a smaller nseg
        const long blocks = ngroups * nseg;
        const long rounds = (blocks + slots - 1) / slots;
        double cost = (double)rounds * (seg + 2 * (K - 1));
        if (blocks < slots) cost *= (double)slots / (double)blocks;
        if (best == 0 || cost < best_cost) {
            best = seg;
            best_cost = cost;
            best_full = 3 * blocks >= slots;
        }
    }
    if (full) *full = best_full;
    return best;
}

hipError_t launch_step2k(bool f32, const void *src, void *dst, const Geo &G, const Phys &P,
                         int K, int seg, hipStream_t st)
{
    const int ns = step2k_strips(G, f32, K);
    const int nb = step2k_blocks(G, f32, K, seg);
    const dim3 grid(nb), block(64 * kXkWaves);
    const bool bnd = geo_bounded(G);
#define LBM_XK_CASE(KK)                                                                       \
    case KK:                                                                                  \
        if (bnd) {                                                                            \
            const hipError_t eb =                                                             \
                f32 ? xkb_launch<float, KK>(grid, block, st, (const float *)src, (float *)dst, \
                                            G, P, ns, seg)                                    \
                    : xkb_launch<double, KK>(grid, block, st, (const double *)src,            \
                                             (double *)dst, G, P, ns, seg);                   \
            if (eb != hipSuccess) return eb;                                                  \
        } else if (f32)                                                                       \
            hipLaunchKernelGGL((k_step2d_xk<float, KK, kXkDepth>), grid, block, 0, st,        \
                               (const float *)src, (float *)dst, G, P, ns, seg);              \
        else                                                                                  \
            hipLaunchKernelGGL((k_step2d_xk<double, KK, kXkDepth>), grid, block, 0, st,       \
                               (const double *)src, (double *)dst, G, P, ns, seg);            \
        break;
    switch (K) {
        LBM_XK_CASE(2)
        LBM_XK_CASE(3)
        LBM_XK_CASE(4)
        LBM_XK_CASE(5)
        LBM_XK_CASE(6)
        LBM_XK_CASE(7)
        LBM_XK_CASE(8)
    default:
        return hipErrorInvalidValue;
    }
#undef LBM_XK_CASE
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(kK1Threads)
    k_step1d_k(const T *__restrict__ src, T *__restrict__ dst, Geo G, Phys P, int K, int nout,
               int whole)
{
    __shared__ T sh[2][4][kK1Threads];
    const int ob = (int)blockIdx.x * nout;
    k1_tile<T, kK1Threads>(src, dst, G, P, K, whole ? 0 : ob - K, ob, nout, sh);
}

// Batched form: workgroup b takes 1D tile b of a table spanning many 1D instances.
template <typename T>
__global__ void __launch_bounds__(kK1Threads)
    k_batch_1k(const InstDev *__restrict__ inst, const K1TileDev *__restrict__ tiles,
               const T *__restrict__ src, T *__restrict__ dst, int K)
{
    __shared__ T sh[2][4][kK1Threads];
    const K1TileDev td = tiles[blockIdx.x];
    const InstDev &I = inst[td.inst];
    k1_tile<T, kK1Threads>(src + I.off, dst + I.off, I.G, I.P, K, td.ob - K, td.ob,
                           kK1Threads - 2 * K, sh);
}

bool step1k_whole(const Geo &G) { return G.bc[0] != BC_PERIODIC && G.nx <= kK1Threads; }

hipError_t launch_step1k(bool f32, const void *src, void *dst, const Geo &G, const Phys &P,
                         int K, hipStream_t st)
{
    // a domain with non-periodic ends that fits one tile: one workgroup, any K
    const int whole = step1k_whole(G) ? 1 : 0;
    if (!whole && 2 * K >= kK1Threads) return hipErrorInvalidValue;
    const int nout = whole ? G.nx : kK1Threads - 2 * K;
    const int nb = whole ? 1 : (G.nx + nout - 1) / nout;
    if (f32)
        hipLaunchKernelGGL(k_step1d_k<float>, dim3(nb), dim3(kK1Threads), 0, st,
                           (const float *)src, (float *)dst, G, P, K, nout, whole);
    else
        hipLaunchKernelGGL(k_step1d_k<double>, dim3(nb), dim3(kK1Threads), 0, st,
                           (const double *)src, (double *)dst, G, P, K, nout, whole);
    return hipGetLastError();
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

// ---- batched launchers -----------------------------------------------------------------
int batch_xk_out(bool f32, int K)
{
    return xk_wo_of(f32, K, false, f32 ? xk_batch_sw<float>() : xk_batch_sw<double>());
}
int batch_xkb_out(bool f32, int K) { return xk_wo_of(f32, K, true); }
int batch_1k_out(int K) { return kK1Threads - 2 * K; }
int batch_xk_waves(bool f32, bool bnd)
{
    const int sw = f32 ? xk_batch_sw<float>() : xk_batch_sw<double>();
    return sw > 1 && !bnd ? 1 : kXkWaves;
}

int batch_xk_per_cu(bool f32, int K)
{
    int n = 0;
    const int bs = 64 * kXkWaves;
    hipError_t e = hipErrorInvalidValue;
#define LBM_BXK_OCC(KK)                                                                       \
    case KK:                                                                                  \
        e = f32 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(                               \
                      &n, k_batch_xk<float, KK, xk_batch_depth<float>()>, bs, 0)              \
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(                               \
                      &n, k_batch_xk<double, KK, xk_batch_depth<double>()>, bs, 0);           \
        break;
    switch (K) {
        LBM_BXK_OCC(2)
        LBM_BXK_OCC(3)
        LBM_BXK_OCC(4)
        LBM_BXK_OCC(5)
        LBM_BXK_OCC(6)
        LBM_BXK_OCC(7)
        LBM_BXK_OCC(8)
    default:
        break;
    }
#undef LBM_BXK_OCC
    return e == hipSuccess ? n : 0;
}

hipError_t launch_batch_xk(bool f32, int K, const InstDev *inst, const XkTileDev *tiles,
                           int ntiles, const void *src, void *dst, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    const dim3 grid(ntiles), block(64 * kXkWaves);
#define LBM_BXK_CASE(KK)                                                                      \
    case KK:                                                                                  \
        if (f32)                                                                              \
            hipLaunchKernelGGL((k_batch_xk<float, KK, xk_batch_depth<float>()>), grid, block, \
                               0, st, inst, tiles, ntiles, (const float *)src, (float *)dst); \
        else                                                                                  \
            hipLaunchKernelGGL((k_batch_xk<double, KK, xk_batch_depth<double>()>), grid, block, \
                               0, st, inst, tiles, ntiles, (const double *)src,               \
                               (double *)dst);                                                \
        break;
    switch (K) {
        LBM_BXK_CASE(2)
        LBM_BXK_CASE(3)
        LBM_BXK_CASE(4)
        LBM_BXK_CASE(5)
        LBM_BXK_CASE(6)
        LBM_BXK_CASE(7)
        LBM_BXK_CASE(8)
    default:
        return hipErrorInvalidValue;
    }
#undef LBM_BXK_CASE
    return hipGetLastError();
}

template <typename T, int KK>
static void bxkb_launch(dim3 grid, dim3 block, hipStream_t st, const InstDev *inst,
                        const XkTileDev *tiles, int ntiles, const T *src, T *dst)
{
    if constexpr (KK <= kXkMaxKBnd)
        hipLaunchKernelGGL((k_batch_xkb<T, KK, kXkbDepth>), grid, block, 0, st, inst, tiles,
                           ntiles, src, dst);
}

hipError_t launch_batch_xkb(bool f32, int K, const InstDev *inst, const XkTileDev *tiles,
                            int ntiles, const void *src, void *dst, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    if (K < 2 || K > kXkMaxKBnd) return hipErrorInvalidValue;
    const dim3 grid(ntiles), block(64 * kXkWaves);
#define LBM_BXKB_CASE(KK)                                                                     \
    case KK:                                                                                  \
        if (f32)                                                                              \
            bxkb_launch<float, KK>(grid, block, st, inst, tiles, ntiles, (const float *)src,  \
                                   (float *)dst);                                             \
        else                                                                                  \
            bxkb_launch<double, KK>(grid, block, st, inst, tiles, ntiles,                     \
                                    (const double *)src, (double *)dst);                      \
        break;
    switch (K) {
        LBM_BXKB_CASE(2)
        LBM_BXKB_CASE(3)
        LBM_BXKB_CASE(4)
        LBM_BXKB_CASE(5)
        LBM_BXKB_CASE(6)
        LBM_BXKB_CASE(7)
        LBM_BXKB_CASE(8)
    default:
        return hipErrorInvalidValue;
    }
#undef LBM_BXKB_CASE
    return hipGetLastError();
}

hipError_t launch_batch_1k(bool f32, int K, const InstDev *inst, const K1TileDev *tiles,
                           int ntiles, const void *src, void *dst, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    if (f32)
        hipLaunchKernelGGL(k_batch_1k<float>, dim3(ntiles), dim3(kK1Threads), 0, st, inst, tiles,
                           (const float *)src, (float *)dst, K);
    else
        hipLaunchKernelGGL(k_batch_1k<double>, dim3(ntiles), dim3(kK1Threads), 0, st, inst, tiles,
                           (const double *)src, (double *)dst, K);
    return hipGetLastError();
}

} // namespace lbm
