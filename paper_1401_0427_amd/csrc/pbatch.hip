// Persistent batched kernel: every step of every instance of a batch in ONE
// launch.  The work of K steps (one pass) is the fused mode's tile tables: 2D
// wave-strip tiles of all-periodic instances, 2D tiles of instances with other
// faces, and 1D LDS tiles (here of 256 nodes, kP1kPerItem to a work item).
// The items of a pass are split into nq = min(kPQueues, grid) claim queues, each
// kind of item into nq contiguous shares (so neighbouring strips of an instance
// share a queue), and workgroup b claims from queue b mod nq in order (its heavy
// 2D tiles first): with eight queues, queue x is served by the workgroups on XCD
// x (workgroups are placed on the XCDs round robin), so the halo columns two
// neighbouring strips both read are fetched once into that XCD's L2.  A pass
// closes when all its items are complete, before the next pass reads what it
// wrote; the buffers swap every pass (pass_claim / pass_complete: the launch
// completes whatever number of its workgroups are resident).  Each tile computes
// exactly what its own launch in the fused mode computes (the same device code),
// so the state equals that of K-step launches, and of single steps, bit for bit.
#include "internal.h"
#include "xk_wave.h"

namespace lbm {

constexpr int kPThreads = 64 * kXkWaves;  // threads per workgroup
constexpr int kP1kPerItem = 16;           // 1D tiles per work item
static_assert(kPQueues == 8, "claim queues: one per XCD");

// Queue x's share of n items split over nq queues: [*start, *start + *count).
__device__ __forceinline__ void pq_share(int n, int nq, int x, int *start, int *count)
{
    const int q = n / nq, r = n % nq;
    *start = x * q + (x < r ? x : r);
    *count = q + (x < r ? 1 : 0);
}

// LDS of the largest tile kind the kernel runs (one array, reused by every item).
template <typename T, int K, bool BND>
constexpr size_t pfused_lds_elems()
{
    constexpr int SW = xk_batch_sw<T>();
    constexpr size_t a = SW > 1 ? (size_t)kXkWaves * xk_wide_rows<T, K, SW>()
                                : (size_t)kXkWaves * xk_lds_elems<T, K>();
    constexpr size_t b = BND ? (size_t)kXkWaves * xkb_lds_elems<T, K>() : 0;
    constexpr size_t c = (size_t)2 * 4 * kPThreads;
    constexpr size_t m = a > b ? a : b;
    return m > c ? m : c;
}

template <typename T, int K, bool BND>
__global__ void __launch_bounds__(kPThreads)
    k_batch_pfused(const InstDev *__restrict__ inst, const XkTileDev *__restrict__ xt, int nxt,
                   const XkTileDev *__restrict__ xbt, int nxbt, const K1TileDev *__restrict__ kt,
                   int nkt, int npasses, T *buf0, T *buf1, int cur, unsigned long long *ctr,
                   int *abort_flag)
{
    constexpr int SW = xk_batch_sw<T>();
    constexpr int D = xk_batch_depth<T>();
    __shared__ __align__(16) T lds[pfused_lds_elems<T, K, BND>()];
    const int wave = (int)(threadIdx.x >> 6);
    const int nk1 = (nkt + kP1kPerItem - 1) / kP1kPerItem;
    const long long nitems = (long long)nxt + nxbt + nk1;
    const int nq = (int)gridDim.x < kPQueues ? (int)gridDim.x : kPQueues;
    const int q = (int)(blockIdx.x % (unsigned)nq);
    int s2, c2, sb, cb, s1, c1;
    pq_share(nxt, nq, q, &s2, &c2);
    pq_share(nxbt, nq, q, &sb, &cb);
    pq_share(nk1, nq, q, &s1, &c1);
    const long long nmine = (long long)c2 + cb + c1;  // this queue's items per pass
    long long pending = -1;
    for (int p = 0; p < npasses; ++p) {
        const bool odd = ((cur + p) & 1) != 0;
        const T *src = odd ? buf1 : buf0;
        T *dst = odd ? buf0 : buf1;
        const long long base = (long long)p * nmine, end = base + nmine;
        int mine = 0;
        for (;;) {
            if (pending < 0) pending = pass_claim(ctr + q);  // (its barrier frees the LDS)
            if (pending >= end) break;                        // kept for a later pass
            const int c = (int)(pending - base);
            pending = -1;
            // the item: this queue's share of 2D tiles, then of bounded tiles, then
            // of 1D items; v numbers it as before (2D, bounded, 1D)
            const int v = c < c2 ? s2 + c : c < c2 + cb ? nxt + sb + (c - c2)
                                                        : nxt + nxbt + s1 + (c - c2 - cb);
            if (v < nxt) {
                const XkTileDev td = xt[v];
                const InstDev &I = inst[td.inst];
                if constexpr (SW > 1) {
                    // one wide strip; every wavefront takes part (workgroup barriers)
                    xk_wave<T, K, D, false, SW>(src + I.off, dst + I.off, I.G, I.P, td.strip0,
                                                td.y0, td.y1, lds, xk_wide_rows<T, K, SW>());
                } else {
                    const int strip = td.strip0 + wave;
                    if (strip < td.nstrips)
                        xk_wave<T, K, D>(src + I.off, dst + I.off, I.G, I.P, strip, td.y0, td.y1,
                                         lds + wave * xk_lds_elems<T, K>());
                }
            } else if (v < nxt + nxbt) {
                if constexpr (BND) {
                    const XkTileDev td = xbt[v - nxt];
                    const InstDev &I = inst[td.inst];
                    const int strip = td.strip0 + wave;
                    if (strip < td.nstrips)
                        xk_wave<T, K, kXkbDepth, true>(src + I.off, dst + I.off, I.G, I.P, strip,
                                                       td.y0, td.y1,
                                                       lds + wave * xkb_lds_elems<T, K>());
                }
            } else {
                const int i0 = (v - nxt - nxbt) * kP1kPerItem;
                const int i1 = min(i0 + kP1kPerItem, nkt);
                for (int i = i0; i < i1; ++i) {
                    const K1TileDev td = kt[i];
                    const InstDev &I = inst[td.inst];
                    k1_tile<T, kPThreads>(src + I.off, dst + I.off, I.G, I.P, K, td.ob - K,
                                          td.ob, kPThreads - 2 * K,
                                          reinterpret_cast<T (*)[4][kPThreads]>(lds));
                }
            }
            ++mine;
        }
        if (pass_complete(ctr + kPQueues, mine, (unsigned long long)((p + 1) * nitems),
                          abort_flag))
            break;
    }
}

int batch_p1k_out(int K) { return kPThreads - 2 * K; }

template <typename T, int K, bool BND>
static int pfused_occ()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch_pfused<T, K, BND>, kPThreads,
                                                     0) != hipSuccess)
        return 0;
    return n;
}

template <typename T, int K, bool BND>
static void pfused_launch(int grid, hipStream_t st, const InstDev *inst, const XkTileDev *xt,
                          int nxt, const XkTileDev *xbt, int nxbt, const K1TileDev *kt, int nkt,
                          int npasses, void *buf0, void *buf1, int cur,
                          unsigned long long *ctr, int *abort_flag)
{
    hipLaunchKernelGGL((k_batch_pfused<T, K, BND>), dim3(grid), dim3(kPThreads), 0, st, inst, xt,
                       nxt, xbt, nxbt, kt, nkt, npasses, (T *)buf0, (T *)buf1, cur, ctr,
                       abort_flag);
}

#define LBM_PF_SWITCH(K, CALL)                                                                \
    switch (K) {                                                                              \
    case 2: CALL(2); break;                                                                   \
    case 3: CALL(3); break;                                                                   \
    case 4: CALL(4); break;                                                                   \
    case 5: CALL(5); break;                                                                   \
    case 6: CALL(6); break;                                                                   \
    case 7: CALL(7); break;                                                                   \
    case 8: CALL(8); break;                                                                   \
    default: break;                                                                           \
    }

// Resident workgroups per compute unit of the persistent kernel (0: unknown K).
int batch_pfused_per_cu(bool f32, int K, bool bnd)
{
    int n = 0;
#define LBM_PF_OCC(KK)                                                                        \
    n = f32 ? (bnd ? pfused_occ<float, KK, true>() : pfused_occ<float, KK, false>())          \
            : (bnd ? pfused_occ<double, KK, true>() : pfused_occ<double, KK, false>())
    LBM_PF_SWITCH(K, LBM_PF_OCC)
#undef LBM_PF_OCC
    return n;
}

hipError_t launch_batch_pfused(bool f32, int K, bool bnd, int grid, const InstDev *inst,
                               const XkTileDev *xt, int nxt, const XkTileDev *xbt, int nxbt,
                               const K1TileDev *kt, int nkt, int npasses, void *buf0,
                               void *buf1, int cur, unsigned long long *ctr,
                               int *abort_flag, hipStream_t st)
{
    if (K < 2 || K > 8 || grid <= 0 || npasses <= 0) return hipErrorInvalidValue;
    if (bnd && K > kXkMaxKBnd) return hipErrorInvalidValue;
#define LBM_PF_LAUNCH(KK)                                                                     \
    if (f32 && bnd)                                                                           \
        pfused_launch<float, KK, true>(grid, st, inst, xt, nxt, xbt, nxbt, kt, nkt, npasses,  \
                                       buf0, buf1, cur, ctr, abort_flag);                     \
    else if (f32)                                                                             \
        pfused_launch<float, KK, false>(grid, st, inst, xt, nxt, xbt, nxbt, kt, nkt, npasses, \
                                        buf0, buf1, cur, ctr, abort_flag);                    \
    else if (bnd)                                                                             \
        pfused_launch<double, KK, true>(grid, st, inst, xt, nxt, xbt, nxbt, kt, nkt, npasses, \
                                        buf0, buf1, cur, ctr, abort_flag);                    \
    else                                                                                      \
        pfused_launch<double, KK, false>(grid, st, inst, xt, nxt, xbt, nxbt, kt, nkt,         \
                                         npasses, buf0, buf1, cur, ctr, abort_flag)
    LBM_PF_SWITCH(K, LBM_PF_LAUNCH)
#undef LBM_PF_LAUNCH
    return hipGetLastError();
}

#undef LBM_PF_SWITCH

} // namespace lbm
