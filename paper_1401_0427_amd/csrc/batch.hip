// Batched form: many independent 1D / 2D problems of uneven size advanced in
// ONE persistent kernel launch.
//
// Work decomposition
//   Every instance is cut into tiles of about `tile_nodes` nodes: runs of
//   consecutive nodes in 1D, bands of whole rows in 2D.  A tile's pull-stream
//   reads only its own nodes and one node (1D) or one row (2D) of each of its
//   two neighbour tiles, so tile t can take step n as soon as t and its
//   neighbours have finished step n-1 -- both for the data it reads and because
//   then nobody still reads the buffer region it overwrites (ping-pong).
//
// Scheduling
//   Work items (step n, tile t) are handed out by one atomic counter in
//   step-major order w = n * T + t.  Every dependency of item w has a smaller
//   index, so it was handed out earlier to a running workgroup; the smallest
//   unfinished item therefore never waits, and the launch cannot deadlock
//   whatever the number of resident workgroups.  There is no grid-wide
//   barrier: fast regions run ahead of slow ones by as many steps as their
//   neighbourhoods allow.  Completion of (n, t) is published by a per-tile
//   counter: one agent-scope release store after a workgroup barrier, and one
//   agent-scope acquire fence after the consumer's relaxed polls succeed.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "lbm.h"
#include "internal.h"

namespace lbm {

struct TileDev {
    int inst;
    int begin, end;  // 1D: node range; 2D: row range
    int nb0, nb1;    // neighbour tiles (-1: none)
};

// Spin (one lane) until tile t has completed n steps.  Polls are relaxed
// agent-scope loads (they read the coherent copy without invalidating any
// cache); the caller issues one acquire fence once every wait has succeeded.
// The wait is bounded: after kSpinLimit polls, or once any workgroup has raised
// the abort flag, it gives up and raises the flag, so every wave of the launch
// always reaches the kernel's exit.  Returns 1 when aborting.

__device__ __forceinline__ int wait_ge(int *done, int t, int n, int *abort_flag)
{
    if (t < 0) return 0;
    for (int k = 0;; ++k) {
        if (__hip_atomic_load(done + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= n) return 0;
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return 1;
        if (k >= kSpinLimit) {
            __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return 1;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// One node of a 2D instance: pull (periodic fast path or boundary rules).
template <typename T>
__device__ __forceinline__ void pull_node2d(const T *__restrict__ s, const InstDev &I, int x, int y,
                                            double *f)
{
    const int nx = I.G.nx, ny = I.G.ny;
    const long ps = I.G.ps;
    const bool interior = x > 0 && x < nx - 1 && y > 0 && y < ny - 1;
    if (I.allper || interior) {
        const long row = (long)y * nx;
        const int xm = x == 0 ? nx - 1 : x - 1;
        const int xp = x == nx - 1 ? 0 : x + 1;
        const long rm = y == 0 ? (long)(ny - 1) * nx : row - nx;
        const long rp = y == ny - 1 ? 0 : row + nx;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T *b = s + (4 * c) * ps;
            f[4 * c + 0] = ld(b + row + xm);
            f[4 * c + 1] = ld(b + ps + rm + x);
            f[4 * c + 2] = ld(b + 2 * ps + row + xp);
            f[4 * c + 3] = ld(b + 3 * ps + rp + x);
        }
    } else {
        pull2d_generic(s, I.G, I.P, x, y, f);
    }
}

// Tiles: with NPP = 2 each thread takes two nodes per pass (both pulls issued
// before either collision) for more loads in flight per thread, at the price
// of registers (occupancy); NPP is a tuning choice.
template <typename T, int NPP>
__device__ __forceinline__ void tile_1d(const T *__restrict__ src, T *__restrict__ dst,
                                        const InstDev &I, int b, int e)
{
    const T *s = src + I.off;
    T *d = dst + I.off;
    const int B = blockDim.x;
    for (int x = b + (int)threadIdx.x; x < e; x += NPP * B) {
        const int x2 = x + B;
        const bool two = NPP == 2 && x2 < e;
        double f[4], g[4];
        pull1d(s, I.G, I.P, x, f);
        if (two) pull1d(s, I.G, I.P, x2, g);
        collide1d<T>(f, I.P);
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) sth<2>(d + pl * I.G.ps + x, f[pl]);
        if (two) {
            collide1d<T>(g, I.P);
#pragma unroll
            for (int pl = 0; pl < 4; ++pl) sth<2>(d + pl * I.G.ps + x2, g[pl]);
        }
    }
}

template <typename T, int NPP>
__device__ __forceinline__ void tile_2d(const T *__restrict__ src, T *__restrict__ dst,
                                        const InstDev &I, int r0, int r1)
{
    const T *s = src + I.off;
    T *d = dst + I.off;
    const int nx = I.G.nx;
    const long ps = I.G.ps;
    const int cnt = (r1 - r0) * nx;
    const int B = blockDim.x;
    for (int k = threadIdx.x; k < cnt; k += NPP * B) {
        const int k2 = k + B;
        const bool two = NPP == 2 && k2 < cnt;
        const int y = r0 + k / nx, x = k - (y - r0) * nx;
        const int y2 = r0 + k2 / nx, x2 = k2 - (y2 - r0) * nx;
        double f[12], g[12];
        pull_node2d(s, I, x, y, f);
        if (two) pull_node2d(s, I, x2, y2, g);
        collide2d<T>(f, I.P);
        T *o = d + (long)y * nx + x;
#pragma unroll
        for (int pl = 0; pl < 12; ++pl) sth<2>(o + pl * ps, f[pl]);
        if (two) {
            collide2d<T>(g, I.P);
            T *o2 = d + (long)y2 * nx + x2;
#pragma unroll
            for (int pl = 0; pl < 12; ++pl) sth<2>(o2 + pl * ps, g[pl]);
        }
    }
}

// 64-bit value of lane 0, as a wave-uniform (scalar) value.
__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long v)
{
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}

// The loop's control flow is uniform by construction: the work index is read
// from LDS into a scalar register (readfirstlane), so the exit is a scalar
// branch, and a barrier separates the release store of one item from the
// dequeue of the next, so no lane-0-only code spans the loop's back edge.
template <typename T, int NPP>
__global__ void __launch_bounds__(512)
    k_batch(const InstDev *__restrict__ inst, const TileDev *__restrict__ tiles, int ntiles,
            unsigned long long nitems, int *done, unsigned long long *next, T *buf0, T *buf1,
            int cur, int *abort_flag)
{
    __shared__ unsigned long long item;
    __shared__ int stop;
    for (;;) {
        if (threadIdx.x == 0) {
            item = atomicAdd(next, 1ull);
            stop = __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        const unsigned long long w = uniform_u64(item);
        if (w >= nitems || __builtin_amdgcn_readfirstlane(stop) != 0) break;
        const int n = (int)(w / (unsigned long long)ntiles);
        const int t = (int)(w - (unsigned long long)n * ntiles);
        const TileDev td = tiles[t];
        if (threadIdx.x == 0) {
            int a = wait_ge(done, t, n, abort_flag);
            if (!a) a = wait_ge(done, td.nb0, n, abort_flag);
            if (!a) a = wait_ge(done, td.nb1, n, abort_flag);
            stop = a;
            // one acquire for all three waits: later loads of this workgroup see
            // the neighbours' step n-1 results
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        if (__builtin_amdgcn_readfirstlane(stop) != 0) break;
        const InstDev I = inst[td.inst];
        const bool odd = ((cur + n) & 1) != 0;
        const T *src = odd ? buf1 : buf0;
        T *dst = odd ? buf0 : buf1;
        if (I.dim == 1)
            tile_1d<T, NPP>(src, dst, I, td.begin, td.end);
        else
            tile_2d<T, NPP>(src, dst, I, td.begin, td.end);
        // the barrier orders every wave's stores before thread 0's agent-scope
        // release (fence cumulativity), which publishes the tile's completion
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_store(done + t, n + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
    }
}

// Unit of the flat and step-synchronous modes: blockDim consecutive flat nodes
// of one instance.
struct UnitDev {
    int inst;
    int k0;  // first flat node (y * nx + x) of the unit in its instance
};

// ---- flat mode -------------------------------------------------------------------
// One ordinary launch per step over every instance: workgroup u takes unit u
// (blockDim consecutive flat nodes y * nx + x of one instance), one node per
// thread, with the same pull / collide code as the tiles above.  The launch
// boundary is the step barrier, so there are no counters, waits or fences;
// the steps are replayed from a captured HIP graph.
template <typename T>
__global__ void __launch_bounds__(512)
    k_batch_flat(const InstDev *__restrict__ inst, const UnitDev *__restrict__ units,
                 const T *__restrict__ src, T *__restrict__ dst)
{
    const UnitDev ud = units[blockIdx.x];
    const InstDev I = inst[ud.inst];
    const int k = ud.k0 + (int)threadIdx.x;
    const int nx = I.G.nx;
    if (k >= nx * I.G.ny) return;
    const long ps = I.G.ps;
    const T *s = src + I.off;
    T *d = dst + I.off;
    if (I.dim == 1) {
        double f[4];
        pull1d(s, I.G, I.P, k, f);
        collide1d<T>(f, I.P);
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) sth<2>(d + pl * ps + k, f[pl]);
        return;
    }
    const int y = k / nx, x = k - y * nx;
    double f[12];
    pull_node2d(s, I, x, y, f);
    collide2d<T>(f, I.P);
    T *o = d + k;
#pragma unroll
    for (int pl = 0; pl < 12; ++pl) sth<2>(o + pl * ps, f[pl]);
}

// ---- step-synchronous mode ------------------------------------------------------------
// Each step's nodes are cut into units of blockDim consecutive (flat) nodes of
// one instance, kSyncUnitsPerItem units to a work item; workgroups claim the
// items of a step in order, so at any moment they work on one contiguous window
// of units (the memory order of the plain kernel) with one node per thread.  A
// step closes when all its items are complete (pass_claim / pass_complete: one
// agent-scope release and one acquire per workgroup per step).  No wait depends
// on a workgroup that has not started, so the grid need not be resident (the
// occupancy query that sizes it ignores the scalar registers, which can admit
// fewer workgroups than it reports); every wait is bounded like the dataflow
// mode's.

// Boundary pulls: the same face rules as the single-grid kernels, with an
// inflow face's equilibrium evaluated in registers.  (A precomputed table
// loaded in the default case of the face switch was miscompiled: the
// control-flow structurizer dropped the table address on one path into that
// case, and the load went through an unassigned register.)
template <typename T>
__device__ __forceinline__ void node_sync(const T *__restrict__ s, T *__restrict__ d,
                                          const InstDev &I, int k)
{
    const Geo &G = I.G;
    const long ps = G.ps;
    if (I.dim == 1) {
        const int x = k;
        double f[4];
        f[0] = x > 0 ? ld(s + x - 1) : pull_face1d(s, G, I.P, 0, 0, x);
        f[2] = x > 0 ? ld(s + 2 * ps + x - 1) : pull_face1d(s, G, I.P, 2, 0, x);
        f[1] = x < G.nx - 1 ? ld(s + ps + x + 1) : pull_face1d(s, G, I.P, 1, 1, x);
        f[3] = x < G.nx - 1 ? ld(s + 3 * ps + x + 1) : pull_face1d(s, G, I.P, 3, 1, x);
        collide1d<T>(f, I.P);
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) sth<2>(d + pl * ps + x, f[pl]);
        return;
    }
    const int nx = G.nx, ny = G.ny;
    const int y = k / nx, x = k - y * nx;
    const long row = (long)y * nx;
    double f[12];
    if (I.allper || (x > 0 && x < nx - 1 && y > 0 && y < ny - 1)) {
        const int xm = x == 0 ? nx - 1 : x - 1;
        const int xp = x == nx - 1 ? 0 : x + 1;
        const long rm = y == 0 ? (long)(ny - 1) * nx : row - nx;
        const long rp = y == ny - 1 ? 0 : row + nx;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T *b = s + (4 * c) * ps;
            f[4 * c + 0] = ld(b + row + xm);
            f[4 * c + 1] = ld(b + ps + rm + x);
            f[4 * c + 2] = ld(b + 2 * ps + row + xp);
            f[4 * c + 3] = ld(b + 3 * ps + rp + x);
        }
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int p = 4 * c;
            f[p] = x > 0 ? ld(s + p * ps + row + x - 1)
                         : pull_face2d(s, G, I.P, p, 0, x, y, x - 1, y);
            f[p + 1] = y > 0 ? ld(s + (p + 1) * ps + row - nx + x)
                             : pull_face2d(s, G, I.P, p + 1, 2, x, y, x, y - 1);
            f[p + 2] = x < nx - 1 ? ld(s + (p + 2) * ps + row + x + 1)
                                  : pull_face2d(s, G, I.P, p + 2, 1, x, y, x + 1, y);
            f[p + 3] = y < ny - 1 ? ld(s + (p + 3) * ps + row + nx + x)
                                  : pull_face2d(s, G, I.P, p + 3, 3, x, y, x, y + 1);
        }
    }
    collide2d<T>(f, I.P);
    T *o = d + row + x;
#pragma unroll
    for (int pl = 0; pl < 12; ++pl) sth<2>(o + pl * ps, f[pl]);
}

// Units of the step-synchronous mode claimed together (one work item).
constexpr int kSyncUnitsPerItem = 8;

template <typename T>
__global__ void __launch_bounds__(512)
    k_batch_sync(const InstDev *__restrict__ inst, const UnitDev *__restrict__ units, int nunits,
                 int nsteps, T *buf0, T *buf1, int cur, unsigned long long *ctr, int *abort_flag)
{
    const long long nitems = (nunits + kSyncUnitsPerItem - 1) / kSyncUnitsPerItem;
    long long pending = -1;
    for (int n = 0; n < nsteps; ++n) {
        const bool odd = ((cur + n) & 1) != 0;
        const T *src = odd ? buf1 : buf0;
        T *dst = odd ? buf0 : buf1;
        const long long base = (long long)n * nitems, end = base + nitems;
        int mine = 0;
        for (;;) {
            if (pending < 0) pending = pass_claim(ctr);
            if (pending >= end) break;  // kept for a later step
            const int u0 = (int)(pending - base) * kSyncUnitsPerItem;
            pending = -1;
            const int u1 = min(u0 + kSyncUnitsPerItem, nunits);
            for (int u = u0; u < u1; ++u) {
                const UnitDev ud = units[u];
                const InstDev I = inst[ud.inst];
                const int k = ud.k0 + (int)threadIdx.x;
                if (k < I.G.nx * I.G.ny)
                    node_sync(src + I.off, dst + I.off, I, k);
            }
            ++mine;
        }
        if (pass_complete(ctr + 1, mine, (unsigned long long)end, abort_flag)) break;
    }
}

// Zero the claim and completion counters (kPersistentCounters: the step-synchronous
// kernel uses the first two, the persistent fused kernel all) and the abort flag of
// a persistent launch (a kernel, so that it can sit in a captured graph).
__global__ void k_batch_sync_reset(unsigned long long *ctr, int *abort_flag)
{
    if (threadIdx.x < kPersistentCounters) ctr[threadIdx.x] = 0ull;
    if (threadIdx.x == 0) *abort_flag = 0;
}

// Zero the per-tile counters and the work counter (a kernel, so that it can sit
// in a captured graph).
__global__ void k_batch_reset(int *done, int ntiles, unsigned long long *next, int *abort_flag)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ntiles) done[i] = 0;
    if (i == 0) {
        *next = 0ull;
        *abort_flag = 0;
    }
}

} // namespace lbm

using namespace lbm;

// ----------------------------------------------------------------- host side ----
static thread_local char b_err[512];
extern "C" const char *lbm_last_error(void);
int lbm_set_error(int code, const char *msg);  // api.hip

static int bfail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(b_err, sizeof b_err, fmt, ap);
    va_end(ap);
    return lbm_set_error(code, b_err);
}

#define BHIP(expr)                                                                        \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return bfail(LBM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

struct lbm_batch {
    std::vector<lbm_instance> inst;
    int storage;
    bool f32;
    void *buf[2];
    int cur;
    long steps;
    hipStream_t st;
    lbm_batch_tuning tune;
    int ntiles;
    InstDev *d_inst;
    TileDev *d_tiles;
    int *d_done;
    unsigned long long *d_next;
    int *d_abort;
    // step-synchronous mode
    UnitDev *d_units;
    int nunits;
    unsigned long long *d_ctr;  // persistent launches: claim counters, completion (kPersistentCounters)
    int grid;
    // fused mode: K steps per launch pair (2D wave-strip tiles + 1D tiles)
    XkTileDev *d_xtiles;
    XkTileDev *d_xbtiles;  // tiles of 2D instances with non-periodic faces
    K1TileDev *d_ktiles;
    int nxtiles, nxbtiles, nktiles;
    int fuse;      // steps per launch
    int xk_seg;    // rows per 2D segment
    long chunk;    // steps per captured graph (flat and fused modes)
    // flat / fused modes: one captured graph of `chunk` steps per starting buffer
    hipGraphExec_t fexec[2];
    // one captured graph per (nsteps, starting buffer); the last one is kept
    hipGraphExec_t gexec;
    long g_nsteps;
    int g_cur;
    hipStream_t cap;
    std::vector<Geo> geo;
    std::vector<Phys> phys;
};

static long round_up(long v, long a) { return ((v + a - 1) / a) * a; }

extern "C" int lbm_batch_layout(lbm_instance *inst, int n, int storage, size_t *bytes,
                                long *nodes)
{
    if (!inst || n <= 0) return bfail(LBM_EINVAL, "need at least one instance");
    if (storage != LBM_F64 && storage != LBM_F32) return bfail(LBM_EINVAL, "bad storage");
    long off = 0, noff = 0;
    for (int i = 0; i < n; ++i) {
        lbm_instance &I = inst[i];
        const bool d1 = I.lattice == LBM_D1Q2x2;
        if (I.lattice != LBM_D1Q2x2 && I.lattice != LBM_D2Q4x3)
            return bfail(LBM_EINVAL, "instance %d: the batched form runs LBM_D1Q2x2 / LBM_D2Q4x3",
                         i);
        if (I.nx < 2 || (d1 ? I.ny != 1 : I.ny < 2))
            return bfail(LBM_EINVAL, "instance %d: bad size %d x %d", i, I.nx, I.ny);
        const long nn = (long)I.nx * I.ny;
        const long ps = round_up(nn, 64);
        I.state_offset = off;
        I.node_offset = noff;
        off += ps * (d1 ? 4 : 12);
        noff += nn;
    }
    if (bytes) *bytes = (size_t)off * (storage == LBM_F32 ? 4 : 8);
    if (nodes) *nodes = noff;
    return LBM_OK;
}

extern "C" void lbm_batch_destroy(lbm_batch *b)
{
    if (!b) return;
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    for (int p = 0; p < 2; ++p)
        if (b->fexec[p]) (void)hipGraphExecDestroy(b->fexec[p]);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    (void)hipFree(b->d_inst);
    (void)hipFree(b->d_tiles);
    (void)hipFree(b->d_done);
    (void)hipFree(b->d_next);
    (void)hipFree(b->d_abort);
    (void)hipFree(b->d_units);
    (void)hipFree(b->d_ctr);
    (void)hipFree(b->d_xtiles);
    (void)hipFree(b->d_xbtiles);
    (void)hipFree(b->d_ktiles);
    delete b;
}

// Rows per 2D segment of the fused mode: one value for every 2D instance, chosen
// like the single-grid launch (tblock.hip, step2k_seg) -- workgroups run in
// rounds of the resident slots and each wavefront runs seg + 2 (K - 1) row
// iterations, so minimise ceil(blocks / slots) * (seg + 2 (K - 1)), a partly
// filled single round counting proportionally longer.
static bool inst_bounded(const lbm_instance &I)
{
    return I.lattice == LBM_D2Q4x3 &&
           !(I.bc[0] == 0 && I.bc[1] == 0 && I.bc[2] == 0 && I.bc[3] == 0);
}

static int fused_seg(bool f32, int K, const std::vector<lbm_instance> &inst, long slots)
{
    int maxny = 0;
    for (const lbm_instance &I : inst)
        if (I.lattice == LBM_D2Q4x3) maxny = std::max(maxny, I.ny);
    if (maxny == 0) return 16;
    if (slots <= 0) return std::min(maxny, 160);
    const int wo = batch_xk_out(f32, K), w = batch_xk_waves(f32, false);
    const int wob = inst.size() && K <= step2k_max_k_bounded() ? batch_xkb_out(f32, K) : wo;
    const int wb = batch_xk_waves(f32, true);
    int best = 0;
    double best_cost = 0.0;
    for (int seg = 16; seg <= maxny; ++seg) {
        long blocks = 0;
        for (const lbm_instance &I : inst) {
            if (I.lattice != LBM_D2Q4x3) continue;
            const bool bnd = inst_bounded(I);
            const int o = bnd ? wob : wo, ww = bnd ? wb : w;
            const long groups = ((I.nx + o - 1) / o + ww - 1) / ww;
            blocks += groups * ((I.ny + seg - 1) / seg);
        }
        const long rounds = (blocks + slots - 1) / slots;
        double cost = (double)rounds * (seg + 2 * (K - 1));
        if (blocks < slots) cost *= (double)slots / (double)blocks;
        if (best == 0 || cost < best_cost) {
            best = seg;
            best_cost = cost;
        }
    }
    return best;
}

extern "C" int lbm_batch_create(const lbm_instance *inst_in, int n, int storage, void *f_a,
                                void *f_b, void *stream, const lbm_batch_tuning *tuning,
                                lbm_batch **out)
{
    if (!out) return bfail(LBM_EINVAL, "null output pointer");
    *out = nullptr;
    if (!inst_in || n <= 0) return bfail(LBM_EINVAL, "need at least one instance");
    if (!f_a || !f_b || f_a == f_b) return bfail(LBM_EINVAL, "need two distinct buffers");
    std::vector<lbm_instance> inst(inst_in, inst_in + n);
    int rc = lbm_batch_layout(inst.data(), n, storage, nullptr, nullptr);
    if (rc) return rc;
    for (int i = 0; i < n; ++i) {
        if (inst[i].state_offset != inst_in[i].state_offset ||
            inst[i].node_offset != inst_in[i].node_offset)
            return bfail(LBM_EINVAL, "instance %d: offsets differ from lbm_batch_layout", i);
        const lbm_instance &I = inst[i];
        if (!(I.lambda > 0) || !(I.s > 0 && I.s < 2) || !(I.g > 0))
            return bfail(LBM_EINVAL, "instance %d: need lambda > 0, s in (0,2), g > 0", i);
        const int nface = I.lattice == LBM_D1Q2x2 ? 2 : 4;
        for (int f = 0; f < nface; ++f) {
            if (I.bc[f] < 0 || I.bc[f] > 3) return bfail(LBM_EINVAL, "instance %d: bad bc", i);
            if ((I.bc[f] == 0) != (I.bc[f ^ 1] == 0))
                return bfail(LBM_EINVAL, "instance %d: periodic faces must be paired", i);
            if (I.bc[f] == LBM_BC_INFLOW && !(I.inflow[f][0] > 0))
                return bfail(LBM_EINVAL, "instance %d: inflow h must be > 0", i);
        }
    }
    lbm_batch_tuning tune = {256, 16384, 0, 1, 0, 0, 0};
    if (tuning) tune = *tuning;
    if (tune.mode < 0 || tune.mode > 4)
        return bfail(LBM_EINVAL, "tuning.mode must be 0 (dataflow), 1 (step-synchronous), 2 "
                                 "(flat), 3 (fused) or 4 (persistent fused)");
    const bool fusedm = tune.mode == 3 || tune.mode == 4;
    if (fusedm) {
        if (tune.fuse_steps < 0 || tune.fuse_steps == 1 || tune.fuse_steps > 8)
            return bfail(LBM_EINVAL, "tuning.fuse_steps must be 0 or in 2 .. 8 (got %d)",
                         tune.fuse_steps);
        for (int i = 0; i < n; ++i) {
            const lbm_instance &I = inst[i];
            if ((long)I.nx * I.ny * (storage == LBM_F32 ? 4 : 8) >= (1L << 31))
                return bfail(LBM_EINVAL, "instance %d: planes of 2 GiB or more (modes 3, 4)",
                             i);
        }
    }
    if (tune.pass_nodes == 0) tune.pass_nodes = 1;
    if (tune.pass_nodes != 1 && tune.pass_nodes != 2)
        return bfail(LBM_EINVAL, "tuning.pass_nodes must be 1 or 2");
    if (tune.block < 64 || tune.block > 512 || tune.block % 64)
        return bfail(LBM_EINVAL, "tuning.block must be a multiple of 64 in [64, 512]");
    if (tune.mode == 0 && tune.tile_nodes < tune.block)
        return bfail(LBM_EINVAL, "tuning.tile_nodes < block");
    if (tune.grid < 0) return bfail(LBM_EINVAL, "tuning.grid must be >= 0");

    lbm_batch *b = new (std::nothrow) lbm_batch();
    if (!b) return bfail(LBM_EDEVICE, "out of host memory");
    b->inst = inst;
    b->storage = storage;
    b->f32 = storage == LBM_F32;
    b->buf[0] = f_a;
    b->buf[1] = f_b;
    b->st = (hipStream_t)stream;
    b->tune = tune;

    std::vector<InstDev> hi(n);
    std::vector<TileDev> ht;
    b->geo.resize(n);
    b->phys.resize(n);
    for (int i = 0; i < n; ++i) {
        const lbm_instance &I = inst[i];
        const int dim = I.lattice == LBM_D1Q2x2 ? 1 : 2;
        InstDev &d = hi[i];
        d.dim = dim;
        d.off = I.state_offset;
        d.G.nx = I.nx;
        d.G.ny = I.ny;
        d.G.ps = round_up((long)I.nx * I.ny, 64);
        for (int f = 0; f < 4; ++f) {
            d.G.bc[f] = (dim == 1 && f >= 2) ? BC_PERIODIC : I.bc[f];
            for (int k = 0; k < 3; ++k) d.G.win[f][k] = I.inflow[f][k];
        }
        d.allper = d.G.bc[0] == 0 && d.G.bc[1] == 0 && d.G.bc[2] == 0 && d.G.bc[3] == 0;
        d.P.c = 0.5 / I.lambda;
        d.P.s = I.s;
        d.P.hg = 0.5 * I.g;
        d.P.g = I.g;
        b->geo[i] = d.G;
        b->phys[i] = d.P;
        // tiles
        const int first = (int)ht.size();
        int nt;
        if (dim == 1) {
            nt = (int)std::max(1L, ((long)I.nx + tune.tile_nodes - 1) / tune.tile_nodes);
            const int per = (I.nx + nt - 1) / nt;
            for (int k = 0; k < nt; ++k) {
                TileDev td;
                td.inst = i;
                td.begin = k * per;
                td.end = std::min(I.nx, (k + 1) * per);
                ht.push_back(td);
            }
        } else {
            const int rows = std::max(1, tune.tile_nodes / I.nx);
            nt = (I.ny + rows - 1) / rows;
            const int per = (I.ny + nt - 1) / nt;
            for (int k = 0; k < nt; ++k) {
                TileDev td;
                td.inst = i;
                td.begin = k * per;
                td.end = std::min(I.ny, (k + 1) * per);
                ht.push_back(td);
            }
        }
        // drop empty tiles that rounding may leave at the end
        while ((int)ht.size() > first + 1 && ht.back().begin >= ht.back().end) ht.pop_back();
        nt = (int)ht.size() - first;
        const bool wrap = dim == 1 ? d.G.bc[0] == BC_PERIODIC : d.G.bc[2] == BC_PERIODIC;
        for (int k = 0; k < nt; ++k) {
            TileDev &td = ht[first + k];
            int a = k - 1, c = k + 1;
            if (a < 0) a = wrap ? nt - 1 : -1;
            if (c >= nt) c = wrap ? 0 : -1;
            td.nb0 = (a < 0 || a == k) ? -1 : first + a;
            td.nb1 = (c < 0 || c == k || c == a) ? -1 : first + c;
        }
    }
    b->ntiles = (int)ht.size();
    // units of the step-synchronous mode: blockDim consecutive flat nodes
    std::vector<UnitDev> hu;
    for (int i = 0; i < n; ++i) {
        const long nn = (long)inst[i].nx * inst[i].ny;
        for (long k0 = 0; k0 < nn; k0 += tune.block) hu.push_back(UnitDev{i, (int)k0});
    }
    if (hu.size() > (size_t)INT32_MAX) {
        lbm_batch_destroy(b);
        return bfail(LBM_EINVAL, "too many units for one launch: raise tuning.block");
    }
    b->nunits = (int)hu.size();
    // fused mode: tile tables of the 2D wave-strip launches (all-periodic instances,
    // and instances with other faces) and of the 1D multi-step launch.  With any
    // 2D instance of the second kind the whole batch takes at most
    // step2k_max_k_bounded() steps per launch, and by default (no fuse_steps)
    // step2k_default_k_bounded().
    std::vector<XkTileDev> hx, hxb;
    std::vector<K1TileDev> hk;
    b->chunk = 32;
    int dev = 0, ncu = 0, per_cu = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (ncu <= 0) ncu = 256;
    if (fusedm) {
        int K = tune.fuse_steps ? tune.fuse_steps : 8;
        bool anyb = false;
        for (int i = 0; i < n; ++i) anyb = anyb || inst_bounded(inst[i]);
        if (anyb && !tune.fuse_steps) K = std::min(K, step2k_default_k_bounded(b->f32));
        if (anyb && K > step2k_max_k_bounded()) K = step2k_max_k_bounded();
        b->fuse = K;
        b->chunk = 2L * K * ((32 + 2 * K - 1) / (2 * K));
        long slots;
        if (tune.mode == 4) {
            // persistent grid: the resident workgroups the occupancy query reports
            // (the launch completes with any grid)
            per_cu = batch_pfused_per_cu(b->f32, K, anyb);
            if (per_cu <= 0) {
                lbm_batch_destroy(b);
                return bfail(LBM_EDEVICE, "no resident workgroup for the persistent kernel");
            }
            long g = (long)ncu * per_cu;
            if (tune.grid > 0 && tune.grid < g) g = tune.grid;
            b->grid = (int)g;
            slots = g;
        } else {
            slots = (long)ncu * batch_xk_per_cu(b->f32, K);
        }
        b->xk_seg = fused_seg(b->f32, K, inst, slots);
        const int wo = batch_xk_out(b->f32, K);
        const int n1 = tune.mode == 4 ? batch_p1k_out(K) : batch_1k_out(K);
        const int wob = anyb ? batch_xkb_out(b->f32, K) : wo;
        for (int i = 0; i < n; ++i) {
            const lbm_instance &I = inst[i];
            if (I.lattice == LBM_D1Q2x2) {
                for (int ob = 0; ob < I.nx; ob += n1) hk.push_back(K1TileDev{i, ob});
                continue;
            }
            const bool bnd = inst_bounded(I);
            const int o = bnd ? wob : wo, w = batch_xk_waves(b->f32, bnd);
            const int ns = (I.nx + o - 1) / o;
            for (int y0 = 0; y0 < I.ny; y0 += b->xk_seg)
                for (int s0 = 0; s0 < ns; s0 += w)
                    (bnd ? hxb : hx)
                        .push_back(XkTileDev{i, s0, ns, y0, std::min(I.ny, y0 + b->xk_seg)});
        }
        if (hx.size() > (size_t)INT32_MAX || hxb.size() > (size_t)INT32_MAX ||
            hk.size() > (size_t)INT32_MAX) {
            lbm_batch_destroy(b);
            return bfail(LBM_EINVAL, "too many tiles for one launch");
        }
    }
    b->nxtiles = (int)hx.size();
    b->nxbtiles = (int)hxb.size();
    b->nktiles = (int)hk.size();

    hipError_t e;
    if ((e = hipMalloc(&b->d_inst, sizeof(InstDev) * n)) != hipSuccess ||
        (e = hipMalloc(&b->d_tiles, sizeof(TileDev) * ht.size())) != hipSuccess ||
        (e = hipMalloc(&b->d_done, sizeof(int) * ht.size())) != hipSuccess ||
        (e = hipMalloc(&b->d_next, sizeof(unsigned long long))) != hipSuccess ||
        (e = hipMalloc(&b->d_abort, sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&b->d_units, sizeof(UnitDev) * hu.size())) != hipSuccess ||
        (e = hipMalloc(&b->d_ctr, kPersistentCounters * sizeof(unsigned long long))) !=
            hipSuccess ||
        (e = hipMalloc(&b->d_xtiles, sizeof(XkTileDev) * std::max<size_t>(1, hx.size()))) !=
            hipSuccess ||
        (e = hipMalloc(&b->d_xbtiles, sizeof(XkTileDev) * std::max<size_t>(1, hxb.size()))) !=
            hipSuccess ||
        (e = hipMalloc(&b->d_ktiles, sizeof(K1TileDev) * std::max<size_t>(1, hk.size()))) !=
            hipSuccess ||
        (!hx.empty() && (e = hipMemcpy(b->d_xtiles, hx.data(), sizeof(XkTileDev) * hx.size(),
                                       hipMemcpyHostToDevice)) != hipSuccess) ||
        (!hxb.empty() && (e = hipMemcpy(b->d_xbtiles, hxb.data(), sizeof(XkTileDev) * hxb.size(),
                                        hipMemcpyHostToDevice)) != hipSuccess) ||
        (!hk.empty() && (e = hipMemcpy(b->d_ktiles, hk.data(), sizeof(K1TileDev) * hk.size(),
                                       hipMemcpyHostToDevice)) != hipSuccess) ||
        (e = hipMemcpy(b->d_units, hu.data(), sizeof(UnitDev) * hu.size(),
                       hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemset(b->d_abort, 0, sizeof(int))) != hipSuccess ||
        (e = hipMemcpy(b->d_inst, hi.data(), sizeof(InstDev) * n, hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(b->d_tiles, ht.data(), sizeof(TileDev) * ht.size(),
                       hipMemcpyHostToDevice)) != hipSuccess) {
        lbm_batch_destroy(b);
        return bfail(LBM_EDEVICE, "batch setup failed: %s", hipGetErrorString(e));
    }
    if ((e = hipGetLastError()) != hipSuccess || (e = hipStreamSynchronize(b->st)) != hipSuccess) {
        lbm_batch_destroy(b);
        return bfail(LBM_EDEVICE, "batch setup failed: %s", hipGetErrorString(e));
    }
    // persistent grid: fill the device
    if (tune.mode >= 2)
        per_cu = 1;  // ordinary launches: one workgroup per unit / tile
    else if (tune.mode == 1 && b->f32)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_sync<float>, tune.block, 0);
    else if (tune.mode == 1)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_sync<double>, tune.block, 0);
    else if (b->f32 && tune.pass_nodes == 2)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<float, 2>, tune.block, 0);
    else if (b->f32)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<float, 1>, tune.block, 0);
    else if (tune.pass_nodes == 2)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<double, 2>, tune.block, 0);
    else
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<double, 1>, tune.block, 0);
    if (per_cu <= 0) per_cu = 1;
    if (tune.mode != 4)
        b->grid = tune.mode == 2 ? b->nunits
                  : tune.mode == 3 ? b->nxtiles + b->nxbtiles + b->nktiles
                                   : (tune.grid > 0 ? tune.grid : ncu * per_cu);
    *out = b;
    return LBM_OK;
}

extern "C" int lbm_batch_init(lbm_batch *b, const double *h0, const double *qx0,
                              const double *qy0)
{
    if (!b) return bfail(LBM_ESTATE, "null batch");
    if (!h0) return bfail(LBM_EINVAL, "null h0");
    unsigned long long *d_speed = nullptr;
    int *d_bad = nullptr;
    BHIP(hipMalloc(&d_speed, sizeof(unsigned long long)));
    hipError_t e = hipMalloc(&d_bad, sizeof(int));
    if (e != hipSuccess) {
        (void)hipFree(d_speed);
        return bfail(LBM_EDEVICE, "hipMalloc failed: %s", hipGetErrorString(e));
    }
    Launch L = {256, 1, 0};
    for (size_t i = 0; i < b->inst.size() && e == hipSuccess; ++i) {
        const lbm_instance &I = b->inst[i];
        const int dim = I.lattice == LBM_D1Q2x2 ? 1 : 2;
        const size_t es = b->f32 ? 4 : 8;
        void *dst = (char *)b->buf[0] + (size_t)I.state_offset * es;
        const long no = I.node_offset;
        e = hipMemsetAsync(d_bad, 0, sizeof(int), b->st);
        if (e == hipSuccess)
            e = launch_init(dim, b->f32, dst, h0 + no, qx0 ? qx0 + no : nullptr,
                            qy0 ? qy0 + no : nullptr, b->geo[i], b->phys[i], L, d_speed, d_bad,
                            b->st);
    }
    int bad = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&bad, d_bad, sizeof bad, hipMemcpyDeviceToHost, b->st);
    if (e == hipSuccess) e = hipStreamSynchronize(b->st);
    (void)hipFree(d_speed);
    (void)hipFree(d_bad);
    if (e != hipSuccess) return bfail(LBM_EDEVICE, "batch init failed: %s", hipGetErrorString(e));
    b->cur = 0;
    b->steps = 0;
    if (bad) return bfail(LBM_EINVAL, "initial fields need finite values and 2^-500 < h < 2^500 "
                                 "everywhere");
    return LBM_OK;
}

static void launch_flat(lbm_batch *b, int cur, hipStream_t st);

// Buffer swaps of nsteps steps: one per step, except in the persistent fused
// mode (one per K-step pass, then one per leftover single step).
static long batch_flips(const lbm_batch *b, long nsteps)
{
    return b->tune.mode == 4 ? nsteps / b->fuse + nsteps % b->fuse : nsteps;
}

static hipError_t enqueue_run(lbm_batch *b, long nsteps, hipStream_t st)
{
    if (b->tune.mode == 4) {
        // one persistent launch of nsteps / K passes, then the leftover steps as
        // single flat launches (the same state bit for bit)
        const long np = nsteps / b->fuse, rem = nsteps % b->fuse;
        int c = b->cur;
        if (np > 0) {
            hipLaunchKernelGGL(k_batch_sync_reset, dim3(1), dim3(64), 0, st, b->d_ctr,
                               b->d_abort);
            hipError_t e = launch_batch_pfused(
                b->f32, b->fuse, b->nxbtiles > 0, b->grid, b->d_inst, b->d_xtiles, b->nxtiles,
                b->d_xbtiles, b->nxbtiles, b->d_ktiles, b->nktiles, (int)np, b->buf[0],
                b->buf[1], c, b->d_ctr, b->d_abort, st);
            if (e != hipSuccess) return e;
            c = (int)((c + np) & 1);
        }
        for (long k = 0; k < rem; ++k) {
            launch_flat(b, c, st);
            c ^= 1;
        }
        return hipGetLastError();
    }
    if (b->tune.mode == 1) {
        hipLaunchKernelGGL(k_batch_sync_reset, dim3(1), dim3(64), 0, st, b->d_ctr, b->d_abort);
        if (b->f32)
            hipLaunchKernelGGL(k_batch_sync<float>, dim3(b->grid), dim3(b->tune.block), 0, st,
                               b->d_inst, b->d_units, b->nunits, (int)nsteps,
                               (float *)b->buf[0], (float *)b->buf[1], b->cur, b->d_ctr,
                               b->d_abort);
        else
            hipLaunchKernelGGL(k_batch_sync<double>, dim3(b->grid), dim3(b->tune.block), 0, st,
                               b->d_inst, b->d_units, b->nunits, (int)nsteps,
                               (double *)b->buf[0], (double *)b->buf[1], b->cur, b->d_ctr,
                               b->d_abort);
        return hipGetLastError();
    }
    const int rb = (b->ntiles + 255) / 256;
    hipLaunchKernelGGL(k_batch_reset, dim3(rb), dim3(256), 0, st, b->d_done, b->ntiles,
                       b->d_next, b->d_abort);
    const unsigned long long nitems = (unsigned long long)nsteps * (unsigned long long)b->ntiles;
#define LBM_BATCH_LAUNCH(TT, NP)                                                               \
    hipLaunchKernelGGL((k_batch<TT, NP>), dim3(b->grid), dim3(b->tune.block), 0, st, b->d_inst, \
                       b->d_tiles, b->ntiles, nitems, b->d_done, b->d_next, (TT *)b->buf[0],    \
                       (TT *)b->buf[1], b->cur, b->d_abort)
    if (b->f32 && b->tune.pass_nodes == 2)
        LBM_BATCH_LAUNCH(float, 2);
    else if (b->f32)
        LBM_BATCH_LAUNCH(float, 1);
    else if (b->tune.pass_nodes == 2)
        LBM_BATCH_LAUNCH(double, 2);
    else
        LBM_BATCH_LAUNCH(double, 1);
#undef LBM_BATCH_LAUNCH
    return hipGetLastError();
}

static void launch_flat(lbm_batch *b, int cur, hipStream_t st)
{
    void *src = b->buf[cur], *dst = b->buf[cur ^ 1];
    if (b->f32)
        hipLaunchKernelGGL(k_batch_flat<float>, dim3(b->nunits), dim3(b->tune.block), 0, st,
                           b->d_inst, b->d_units, (const float *)src, (float *)dst);
    else
        hipLaunchKernelGGL(k_batch_flat<double>, dim3(b->nunits), dim3(b->tune.block), 0, st,
                           b->d_inst, b->d_units, (const double *)src, (double *)dst);
}

// K steps of every instance from buffer cur into the other: the 2D wave-strip
// tiles (all-periodic instances, then those with other faces), then the 1D tiles
// (independent instances; one ordered sequence of launches).
static hipError_t launch_fused(lbm_batch *b, int cur, hipStream_t st)
{
    const void *src = b->buf[cur];
    void *dst = b->buf[cur ^ 1];
    hipError_t e = launch_batch_xk(b->f32, b->fuse, b->d_inst, b->d_xtiles, b->nxtiles, src, dst,
                                   st);
    if (e == hipSuccess)
        e = launch_batch_xkb(b->f32, b->fuse, b->d_inst, b->d_xbtiles, b->nxbtiles, src, dst,
                             st);
    if (e == hipSuccess)
        e = launch_batch_1k(b->f32, b->fuse, b->d_inst, b->d_ktiles, b->nktiles, src, dst, st);
    return e;
}

// Flat and fused modes: whole chunks of b->chunk steps (an even number of
// launches, so the chunk starts and ends on the same buffer) replay one captured
// graph per starting buffer; the remaining steps are launched directly (whole
// fused launches, then single flat steps, which give the same state bit for bit).
static int run_flat(lbm_batch *b, long nsteps)
{
    const bool fused = b->tune.mode == 3;
    const long per = fused ? b->fuse : 1;
    long left = nsteps;
    if (b->tune.direct) {
        // no graph: every launch directly on the stream
        for (; fused && left >= per; left -= per) {
            BHIP(launch_fused(b, b->cur, b->st));
            b->cur ^= 1;
            b->steps += per;
        }
        for (; left > 0; --left) {
            launch_flat(b, b->cur, b->st);
            BHIP(hipGetLastError());
            b->cur ^= 1;
            ++b->steps;
        }
        return LBM_OK;
    }
    if (left >= b->chunk && !b->fexec[b->cur]) {
        if (!b->cap) BHIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        BHIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
        hipError_t le = hipSuccess;
        for (long k = 0; k < b->chunk / per && le == hipSuccess; ++k) {
            const int c = (int)((b->cur + k) & 1);
            if (fused)
                le = launch_fused(b, c, b->cap);
            else
                launch_flat(b, c, b->cap);
        }
        if (le == hipSuccess) le = hipGetLastError();
        hipError_t ee = hipStreamEndCapture(b->cap, &g);
        if (le != hipSuccess || ee != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return bfail(LBM_EDEVICE, "batch graph capture failed: %s",
                         hipGetErrorString(le != hipSuccess ? le : ee));
        }
        hipError_t ie = hipGraphInstantiate(&b->fexec[b->cur], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) {
            b->fexec[b->cur] = nullptr;
            return bfail(LBM_EDEVICE, "batch graph instantiate failed: %s", hipGetErrorString(ie));
        }
    }
    for (; left >= b->chunk; left -= b->chunk) {
        BHIP(hipGraphLaunch(b->fexec[b->cur], b->st));
        b->steps += b->chunk;
    }
    for (; fused && left >= per; left -= per) {
        BHIP(launch_fused(b, b->cur, b->st));
        b->cur ^= 1;
        b->steps += per;
    }
    for (; left > 0; --left) {
        launch_flat(b, b->cur, b->st);
        BHIP(hipGetLastError());
        b->cur ^= 1;
        ++b->steps;
    }
    return LBM_OK;
}

extern "C" int lbm_batch_run(lbm_batch *b, long nsteps)
{
    if (!b) return bfail(LBM_ESTATE, "null batch");
    if (nsteps < 0 || nsteps > (1L << 30)) return bfail(LBM_EINVAL, "bad nsteps");
    if (b->tune.mode == 2 || b->tune.mode == 3) return run_flat(b, nsteps);
    if (nsteps == 0) return LBM_OK;
    if (b->tune.direct) {
        BHIP(enqueue_run(b, nsteps, b->st));
        b->steps += nsteps;
        b->cur = (int)((b->cur + batch_flips(b, nsteps)) & 1);
        return LBM_OK;
    }
    if (!b->gexec || b->g_nsteps != nsteps || b->g_cur != b->cur) {
        if (b->gexec) {
            (void)hipGraphExecDestroy(b->gexec);
            b->gexec = nullptr;
        }
        if (!b->cap) BHIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        BHIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
        hipError_t le = enqueue_run(b, nsteps, b->cap);
        hipError_t ee = hipStreamEndCapture(b->cap, &g);
        if (le != hipSuccess || ee != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return bfail(LBM_EDEVICE, "batch graph capture failed: %s",
                         hipGetErrorString(le != hipSuccess ? le : ee));
        }
        hipError_t ie = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) {
            b->gexec = nullptr;
            return bfail(LBM_EDEVICE, "batch graph instantiate failed: %s", hipGetErrorString(ie));
        }
        b->g_nsteps = nsteps;
        b->g_cur = b->cur;
    }
    BHIP(hipGraphLaunch(b->gexec, b->st));
    b->steps += nsteps;
    b->cur = (int)((b->cur + batch_flips(b, nsteps)) & 1);
    return LBM_OK;
}

extern "C" int lbm_batch_check(lbm_batch *b)
{
    if (!b) return bfail(LBM_ESTATE, "null batch");
    int flag = 0;
    BHIP(hipMemcpyAsync(&flag, b->d_abort, sizeof flag, hipMemcpyDeviceToHost, b->st));
    BHIP(hipStreamSynchronize(b->st));
    if (flag)
        return bfail(LBM_EDEVICE, "batched run aborted: a wait of the persistent launch (tile "
                                  "dependency or grid barrier) did not end within its limit "
                                  "(state is invalid)");
    return LBM_OK;
}

extern "C" int lbm_batch_moments(lbm_batch *b, double *h, double *qx, double *qy)
{
    if (!b) return bfail(LBM_ESTATE, "null batch");
    const size_t es = b->f32 ? 4 : 8;
    for (size_t i = 0; i < b->inst.size(); ++i) {
        const lbm_instance &I = b->inst[i];
        const int dim = I.lattice == LBM_D1Q2x2 ? 1 : 2;
        const void *s = (const char *)b->buf[b->cur] + (size_t)I.state_offset * es;
        const long no = I.node_offset;
        BHIP(launch_moments(dim, b->f32, s, h ? h + no : nullptr, qx ? qx + no : nullptr,
                            (qy && dim == 2) ? qy + no : nullptr, nullptr, b->geo[i], b->st,
                            nullptr));
    }
    return LBM_OK;
}

extern "C" int lbm_batch_current(lbm_batch *b, void **state, long *steps_done)
{
    if (!b) return bfail(LBM_ESTATE, "null batch");
    if (state) *state = b->buf[b->cur];
    if (steps_done) *steps_done = b->steps;
    return LBM_OK;
}

// Number of work tiles and workgroups per launch (for tuning reports).
extern "C" int lbm_batch_info(lbm_batch *b, int *ntiles, int *grid)
{
    if (!b) return bfail(LBM_ESTATE, "null batch");
    if (ntiles)
        *ntiles = b->tune.mode == 0 ? b->ntiles
                  : b->tune.mode >= 3 ? b->nxtiles + b->nxbtiles + b->nktiles
                                      : b->nunits;
    if (grid) *grid = b->grid;
    return LBM_OK;
}
