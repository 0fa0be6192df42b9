// Internal declarations shared by the host-side sources of liblbm.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "lbm_device.h"

namespace lbm {

// Constants of the rest-population schemes (D1Q3Q2 / D2Q5Q4Q4) with MRT.
struct Mrt {
    double lam, il;   // lambda and 1 / lambda
    double a, aK;     // rest weight and a K, K = 1 / (2 g)
    double g, hg, c;  // g, g / 2, 1 / (2 lambda)
    double rate[10];  // relaxation rates of the non-conserved moments
};

// One instance of the batched form: geometry, physics and the element offset of
// its planes in the batch buffers.
struct InstDev {
    int dim;
    int allper;  // all faces periodic
    long off;    // element offset of the instance's planes in the batch buffer
    Geo G;
    Phys P;
};

// Tile of the batched multi-step launch of 2D instances: strips [strip0,
// strip0 + waves) (of nstrips) of instance inst, output rows [y0, y1).
struct XkTileDev {
    int inst;
    int strip0, nstrips;
    int y0, y1;
};

// Tile of the batched multi-step launch of 1D instances: output nodes [ob, ob +
// 1024 - 2K) of instance inst.
struct K1TileDev {
    int inst;
    int ob;
};

// Polls at most of a bounded wait in a persistent launch.
constexpr int kSpinLimit = 1 << 22;
// Claim queues of the persistent fused batch kernel (one per XCD); its counters are
// kPQueues claim counters followed by the completion counter.
constexpr int kPQueues = 8;
constexpr int kPersistentCounters = kPQueues + 1;

// Work distribution of a persistent launch that advances in passes (one step, or
// K steps) over nitems work items each.  A 64-bit claim counter hands out item
// indices in order (pass p owns [p nitems, (p + 1) nitems)); a workgroup that
// finds the pass exhausted adds the number of items it completed to a 64-bit
// completion counter and waits until the pass's total is reached.  No wait
// depends on a workgroup that has not started, so a launch completes whatever
// number of its workgroups are resident at once (residency decides only the
// speed); an index claimed beyond the pass is kept for the pass it belongs to.

// Claim the next index (the same value on every lane of the workgroup).  The
// leading barrier also ends every wave's use of the LDS by the previous item.
__device__ __forceinline__ long long pass_claim(unsigned long long *next)
{
    __shared__ unsigned long long s_claim;
    __syncthreads();
    if (threadIdx.x == 0)
        s_claim = __hip_atomic_fetch_add(next, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const unsigned long long v = s_claim;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

// Report `mine` completed items and wait until `target` items in all are
// complete.  The workgroup barrier orders every wave's stores before thread 0's
// agent-scope release (the fetch-add; fence cumulativity); thread 0 then polls
// with relaxed loads and issues one agent-scope acquire for the workgroup.  The
// wait is bounded: after kSpinLimit polls, or once any workgroup has raised the
// abort flag, it raises the flag and gives up.  Returns nonzero (the same on
// every lane of the workgroup) when the launch is aborting.
__device__ __forceinline__ int pass_complete(unsigned long long *done, int mine,
                                             unsigned long long target, int *abort_flag)
{
    __shared__ int s_stop;
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(done, (unsigned long long)mine, __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
        int a = 0;
        for (int it = 0;; ++it) {
            if (__hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target)
                break;
            if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                a = 1;
                break;
            }
            if (it >= kSpinLimit) {
                __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                a = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_stop = a;
    }
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(s_stop);
}

// Launch shape of the plain forward / adjoint kernels.
struct Launch {
    int block;  // threads per workgroup
    int npt;    // nodes per thread along x
    int hints;  // bit 0 non-temporal loads, bit 1 non-temporal stores, bit 2 no XCD remap
};

// Kernel launchers (each returns the hipError_t of the launch).
hipError_t launch_init(int dim, bool f32, void *dst, const double *h0, const double *qx0,
                       const double *qy0, const Geo &G, const Phys &P, const Launch &L,
                       unsigned long long *speed_bits, int *bad, hipStream_t st);
hipError_t launch_step(int dim, bool f32, const void *src, void *dst, const Geo &G,
                       const Phys &P, const Launch &L, hipStream_t st);
hipError_t launch_moments(int dim, bool f32, const void *state, double *h, double *qx,
                          double *qy, double *partials, const Geo &G, hipStream_t st,
                          int *nblocks_out);
hipError_t launch_sum(const double *in, long n, int stride, int ncomp, double *out,
                      hipStream_t st);
hipError_t launch_check(int dim, bool f32, const void *state, const Geo &G, int *flag,
                        hipStream_t st);
int moments_blocks(const Geo &G);

// f32: state storage float; a32: adjoint storage float (double otherwise; a float
// adjoint needs a float state).  side: adjoint_side_len(G) x 4 faces x 3 doubles of
// scratch for the Neumann faces (may be null when no face is Neumann).
hipError_t launch_adjoint(int dim, bool f32, bool a32, const void *un, const void *lam1,
                          void *lam0, double *partials, double *side, const Geo &G,
                          const Phys &P, hipStream_t st);
int adjoint_side_len(const Geo &G);
long adjoint_blocks(const Geo &G);
hipError_t launch_adjoint_terminal(int dim, bool f32, const double *dLdh, void *lam,
                                   const Geo &G, hipStream_t st);
hipError_t launch_adjoint_grad_w0(int dim, bool f32, const void *lam0, const double *h0,
                                  const double *qx0, const double *qy0, double *gh, double *gqx,
                                  double *gqy, const Geo &G, const Phys &P, hipStream_t st);

int step2x_blocks(const Geo &G, int seg);
// 1D K-step launch: tiles of kK1Threads nodes with 2 K halo nodes (K < 512), or,
// for a domain with non-periodic ends of at most kK1Threads nodes (step1k_whole),
// one whole-domain tile and any K.
bool step1k_whole(const Geo &G);
hipError_t launch_step1k(bool f32, const void *src, void *dst, const Geo &G, const Phys &P,
                         int K, hipStream_t st);
hipError_t launch_step2x(bool f32, const void *src, void *dst, const Geo &G, const Phys &P,
                         int seg, hipStream_t st);
int step2k_blocks(const Geo &G, bool f32, int K, int seg);
int step2k_seg(const Geo &G, bool f32, int K, int min_seg, bool *full, long *slots_out);
int step2k_max_k_bounded();  // steps per launch at most with non-periodic faces
int step2k_default_k_bounded(bool f32);  // and by default

// Batched multi-step launches (tblock.hip).
int batch_xk_out(bool f32, int K);   // output columns per strip
int batch_xkb_out(bool f32, int K);  // the same, instances with non-periodic faces
int batch_1k_out(int K);            // output nodes per 1D tile
int batch_xk_waves(bool f32, bool bnd);  // strips per workgroup (bnd: non-periodic faces)
int batch_xk_per_cu(bool f32, int K);
hipError_t launch_batch_xk(bool f32, int K, const InstDev *inst, const XkTileDev *tiles,
                           int ntiles, const void *src, void *dst, hipStream_t st);
hipError_t launch_batch_xkb(bool f32, int K, const InstDev *inst, const XkTileDev *tiles,
                            int ntiles, const void *src, void *dst, hipStream_t st);
hipError_t launch_batch_1k(bool f32, int K, const InstDev *inst, const K1TileDev *tiles,
                           int ntiles, const void *src, void *dst, hipStream_t st);

// Persistent batched launch (pbatch.hip): npasses passes of K steps over every
// tile of the three tables (2D all-periodic, 2D with other faces, 1D) in one
// launch; ctr = {claim counter, completion counter}, zero before the launch.
int batch_p1k_out(int K);  // output nodes per 1D tile of the persistent launch
int batch_pfused_per_cu(bool f32, int K, bool bnd);
hipError_t launch_batch_pfused(bool f32, int K, bool bnd, int grid, const InstDev *inst,
                               const XkTileDev *xt, int nxt, const XkTileDev *xbt, int nxbt,
                               const K1TileDev *kt, int nkt, int npasses, void *buf0,
                               void *buf1, int cur, unsigned long long *ctr, int *abort_flag,
                               hipStream_t st);
hipError_t launch_step2k(bool f32, const void *src, void *dst, const Geo &G, const Phys &P,
                         int K, int seg, hipStream_t st);
hipError_t launch_entropy(int dim, bool f32, const void *state, const Geo &G, double lambda,
                          double g, double *h_node, double *partials, hipStream_t st,
                          int *nblocks_out);

hipError_t launch_init_rest(int dim, bool f32, void *dst, const double *h0, const double *qx0,
                            const double *qy0, const Geo &G, const Mrt &M,
                            unsigned long long *speed_bits, int *bad, hipStream_t st);
hipError_t launch_step_rest(int dim, bool f32, const void *src, void *dst, const Geo &G,
                            const Mrt &M, hipStream_t st);
hipError_t launch_moments_rest(int dim, bool f32, const void *state, double *h, double *qx,
                               double *qy, double *partials, int *flag, const Geo &G,
                               hipStream_t st, int *nblocks_out);

} // namespace lbm
