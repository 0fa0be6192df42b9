// Multi-step launches of the rest-population lattices (csrc/mrt.hip), outside the
// hot path's wave-strip kernels.
#pragma once
#include "internal.h"

namespace lbm {

// D2Q5Q4Q4 on all-periodic grids, K = 2 .. kMaxFuseRest2d steps per launch
// (one wavefront per 64-column strip, four to a 256-thread workgroup, segments of
// `seg` rows; bitwise equal to K single steps).  rest2k_seg: the segment length
// for the device's resident workgroups (0 if it cannot be queried), slots_out the
// resident workgroups; rest2k_blocks: workgroups of one launch.
constexpr int kMaxFuseRest2d = 6;
constexpr int kRestMinSeg = 16;
int rest2k_seg(const Geo &G, bool f32, int K, long *slots_out);
long rest2k_blocks(const Geo &G, int K, int seg);
hipError_t launch_step_rest2k(bool f32, const void *src, void *dst, const Geo &G, const Mrt &M,
                              int K, int seg, hipStream_t st);
// D1Q3Q2, K steps per launch: tiles of kK1Threads nodes with 2 K halo nodes (K < 512),
// or one whole-domain tile for any K (step1k_whole); bitwise equal to K single steps.
hipError_t launch_step_rest1k(bool f32, const void *src, void *dst, const Geo &G, const Mrt &M,
                              int K, hipStream_t st);

} // namespace lbm
