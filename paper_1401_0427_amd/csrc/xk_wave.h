// Device code of the multi-step launches: the wave-strip march of K time levels
// over a 2D column strip (all-periodic and bounded forms) and the LDS tile of K
// steps over 1D nodes.  Included by the kernels that launch them one tile per
// workgroup and by the persistent batched kernel.
#pragma once

#include "internal.h"

namespace lbm {

// ---- 2D: K steps per launch, one wavefront per column strip ------------------------
// Each wavefront works alone (no LDS, no barrier): lane l holds column
// x0 - (K - 1) + l and the wavefront marches up a segment of rows with the K
// time levels skewed by one row: in iteration i it computes level 1 at row i,
// level 2 at row i - 1, ..., level K at row i - K + 1.  Level k + 1 at row r
// pulls from level k: e2 planes of row r - 1 and e4 planes of row r + 1 from
// the lane's own registers, e1 planes of row r from lane l - 1 and e3 planes
// from lane l + 1 (cross-lane permutes).  Level 1 pulls straight from the
// level-n state in memory.  Each level loses one lane at each end of the
// wavefront, so a strip yields 64 - 2 (K - 1) output columns; the segment is
// extended by K - 1 rows at each end for the same reason.  Intermediate levels
// are rounded to the storage type (as a store and reload would round them), and
// the per-node arithmetic is the one-step kernel's, so K steps in one launch
// equal K single steps bit for bit.  The next row's level-n pulls are issued
// before the current row is computed, so loads overlap the arithmetic.  The row
// loop is unrolled by two with the roles of the row registers swapped, so no
// register is copied from one row to the next; plane addresses are a uniform
// base plus a 32-bit byte offset (planes below 2 GiB).
// Rows of level-n pulls in flight ahead of the row being computed.  Measured at
// 4096^2, alternating runs on one device: FP64 K = 8 174-176 GLUPS with one row,
// 171-173 with two; FP32 (256-lane strips, K = 8) 223 either way, with 154
// instead of 178 registers.
// FP64 launches of at least kXkLdsMinK steps exchange the e1 / e3 planes of
// their first kXkLdsLevelsF64 intermediate levels through a per-wavefront LDS row
// instead of cross-lane permutes into registers; 0 levels = off.  At K = 8 this
// takes the kernel from 332 registers (one wavefront per SIMD) to 231 (two):
// 171 vs 157 GLUPS at 4096^2 (4, 5 or 6 levels alike; 6 uses 72 KiB of LDS per
// workgroup, two workgroups per compute unit).  At K = 6 the permutes hold 256
// registers plus spills (one wavefront per SIMD) and the LDS rows 170 (two):
// 0.710 against 0.716 ms per 4096^2 launch; at K = 4 and 5 the permute form,
// already at two wavefronts per SIMD, is the faster one (0.725 / 0.734 ms against
// 0.734 / 0.747 with LDS rows at three).
constexpr int kXkLdsLevelsF64 = 6;
// LDS exchange levels read one level ahead, for FP32 launches of at most this
// many steps (0: never).  Measured at 2048^2, FP32 K = 6: 159-160 GLUPS against
// 151; FP32 K = 8 at 4096^2: 221 against 224; FP64 K = 8 unchanged (177).
constexpr int kXkLdsPrefetchF32MaxK = 6;
constexpr int kXkLdsMinK = 6;
constexpr int kXkLdsLevelsF32 = 0;  // the same for FP32 launches (0 = off)
// Output strips start and end on this many bytes (0: no alignment), and the
// stores are non-temporal (1) or not (0), per storage type.  Measured at 4096^2:
// FP64 -- 64-byte strips with non-temporal stores (94 vs 77 GLUPS unaligned);
// FP32 -- unaligned strips with ordinary stores, whose partly written segments
// at strip edges merge in L2 (140 vs 122 GLUPS for 64-byte strips).
constexpr int kXkAlignF64 = 64;
constexpr int kXkNtF64 = 1;
constexpr int kXkAlignF32 = 0;
constexpr int kXkNtF32 = 0;
constexpr int kXkWaves = 4;  // wavefronts per workgroup
// Wide strips, per storage type: the all-periodic single-grid launch gives each
// workgroup one strip of 64 x kXkWaves lanes (0: one 64-lane strip per
// wavefront).  Wavefronts then meet inside a strip and exchange their edge
// lanes' e1 / e3 planes through LDS, with one workgroup barrier per row; the
// halo lanes recomputed per strip drop from 2 (K - 1) per 64 to 2 (K - 1) per
// 64 x kXkWaves.  Measured at 4096^2, alternating runs on one device: FP32 K = 6
// 208 GLUPS with 64-lane strips, 219-221 wide, K = 8 wide 222-224; FP64 no gain
// (K = 8: 158-164 wide against 163-166, K = 7: 134-149 against 143).
constexpr int kXkWideF64 = 0;
constexpr int kXkWideF32 = 1;
template <typename T>
constexpr int xk_sw()
{
    return (sizeof(T) == 8 ? kXkWideF64 : kXkWideF32) ? kXkWaves : 1;
}
constexpr int kXkDepth = 1;  // rows of level-n pulls in flight
// Wide strips in the batched launch (all-periodic instances), per storage type as
// for single grids: 1 = the storage type's xk_sw, 0 = 64-lane strips.  The
// 256-instance manifest (FP32, K = 8, fused against flat mode bit for bit): 184
// GLUPS with 256-lane strips, 170 with 64-lane strips.
constexpr int kXkBatchWide = 1;
template <typename T>
constexpr int xk_batch_sw()
{
    return kXkBatchWide ? xk_sw<T>() : 1;
}
// Rows of level-n pulls in flight in the batched launch, per storage type.  The
// same manifest, FP32: 64-lane strips 164-172 GLUPS with two rows, 155 with one;
// 256-lane strips 184 with one row (154 registers, three wavefronts per SIMD),
// 179 with two (183 registers).
constexpr int kXkBatchDepthF64 = 2;
constexpr int kXkBatchDepthF32 = 1;
template <typename T>
constexpr int xk_batch_depth()
{
    return sizeof(T) == 4 ? kXkBatchDepthF32 : kXkBatchDepthF64;
}

// Workgroup b runs on XCD b % 8 (round-robin dispatch).  Give XCD x the
// contiguous tile range [x q + min(x, r), ...) of q + (x < r) tiles (q, r =
// ntiles / 8, ntiles % 8): neighbouring strips then share one XCD's L2, so the
// halo columns two strips both read are fetched from memory once.  A bijection
// of [0, ntiles) for any ntiles.
__device__ __forceinline__ int xk_tile(int b, int ntiles, bool remap)
{
    if (!remap) return b;
    const int x = b & 7, k = b >> 3, q = ntiles >> 3, r = ntiles & 7;
    return x * q + (x < r ? x : r) + k;
}

// Value of lane l - 1 (shift 1) or lane l + 1 (shift -1); the end lanes get an
// arbitrary lane's value (they are outside the valid range of the next level).
__device__ __forceinline__ float xk_from(float v, int lane, int shift)
{
    const int src = (lane - shift) & 63;
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}
__device__ __forceinline__ double xk_from(double v, int lane, int shift)
{
    const int src = ((lane - shift) & 63) << 2;
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(src, (int)(b & 0xffffffffLL));
    const int hi = __builtin_amdgcn_ds_bpermute(src, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// The same exchange through DPP wave shifts (a VALU move, no LDS access):
// xk_shr gives lane l the value of lane l - 1, xk_shl that of lane l + 1; the
// end lanes receive 0.
template <int CTRL>
__device__ __forceinline__ float xk_dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double xk_dpp(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename T>
__device__ __forceinline__ T xk_shr(T v)
{
    return xk_dpp<0x138>(v);  // wave_shr:1
}
template <typename T>
__device__ __forceinline__ T xk_shl(T v)
{
    return xk_dpp<0x130>(v);  // wave_shl:1
}
template <typename T>
__device__ __forceinline__ T xk_xch(T v, int lane, int shift)
{
    return xk_from(v, lane, shift);
}

template <typename T>
__device__ __forceinline__ T xk_at(const T *base, unsigned off)
{
    return *(const T *)((const char *)base + off);
}

// Byte offsets (within a plane) of the level-n pulls of one level-1 node.
struct XkOff {
    unsigned e1, e2, e3, e4;
};

template <typename T>
__device__ __forceinline__ XkOff xk_offsets(int r, int nx, int ny, int xm, int xw, int xp)
{
    const unsigned row = (unsigned)r * (unsigned)nx;
    const unsigned rm = r == 0 ? (unsigned)(ny - 1) * (unsigned)nx : row - nx;
    const unsigned rp = r == ny - 1 ? 0u : row + nx;
    return XkOff{(row + xm) * (unsigned)sizeof(T), (rm + xw) * (unsigned)sizeof(T),
                 (row + xp) * (unsigned)sizeof(T), (rp + xw) * (unsigned)sizeof(T)};
}

template <typename T>
__device__ __forceinline__ void xk_load(const T *__restrict__ src, long ps, const XkOff &o, T *f)
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        f[4 * c + 0] = xk_at(src + (4 * c + 0) * ps, o.e1);
        f[4 * c + 1] = xk_at(src + (4 * c + 1) * ps, o.e2);
        f[4 * c + 2] = xk_at(src + (4 * c + 2) * ps, o.e3);
        f[4 * c + 3] = xk_at(src + (4 * c + 3) * ps, o.e4);
    }
}

// ---- grids with non-periodic faces ------------------------------------------------
// The face rules are those of the one-step kernel (pull_face2d): a pull from
// outside the grid through face f takes, at the boundary node itself,
//   Neumann -- the same population;
//   wall    -- the opposite population, negated for the normal momentum
//              (qx on the x faces, qy on the y faces);
//   inflow  -- the equilibrium of the face's prescribed state (in double, not
//              rounded to the storage type).
// Level 1 applies them to the level-n state in memory; every further level to
// the boundary node's own values of the previous level.  Lanes and rows outside
// the grid read clamped addresses: their values are never pulled by a node of
// the grid (its pulls through the faces are replaced), so they never reach a
// stored value.
struct XkBnd {
    int kx0, kx1, ky0, ky1;  // face rules (BC_PERIODIC: the axis wraps)
    double in1[3], in3[3];   // inflow equilibria of the e1 planes (x-), e3 planes (x+)
    double in2[3], in4[3];   // of the e2 planes (y-), e4 planes (y+)
};

// A value equal on every lane, moved to scalar registers (the face values are
// computed from kernel arguments, so every lane holds the same bits).
__device__ __forceinline__ double xk_uniform(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename T>
__device__ __forceinline__ XkBnd xk_bnd(const Geo &G, const Phys &P)
{
    XkBnd B;
    B.kx0 = G.bc[0];
    B.kx1 = G.bc[1];
    B.ky0 = G.bc[2];
    B.ky1 = G.bc[3];
    double e[12];
    const int jp[4] = {0, 2, 1, 3};  // plane in a family pulled through face f
    double *dst[4] = {B.in1, B.in3, B.in2, B.in4};
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        feq2d<T>(G.win[f][0], G.win[f][1], G.win[f][2], P, e);
#pragma unroll
        for (int c = 0; c < 3; ++c) dst[f][c] = xk_uniform(e[4 * c + jp[f]]);
    }
    return B;
}

__device__ __forceinline__ int xk_clampw(int v, int n, bool per)
{
    return per ? ((v % n) + n) % n : min(max(v, 0), n - 1);
}

// Level-n pulls of the level-1 nodes of row i (unwrapped) on a grid with
// non-periodic faces; xm / xw / xp: the lane's column and its neighbours,
// clamped to the grid on a non-periodic x axis.  Clamped rows and columns give a
// face node its own population, the Neumann rule; a y wall takes the opposite
// plane of the node's own row (uniform over the wavefront).  The x wall, the
// sign flips and the inflow values are applied where the row is consumed.
template <typename T>
__device__ __forceinline__ void xk_load_clamp(const T *__restrict__ src, long ps, const Geo &G,
                                              const XkBnd &B, int i, int xm, int xw, int xp,
                                              T *f)
{
    const int nx = G.nx, ny = G.ny;
    const bool pery = B.ky0 == BC_PERIODIC;
    const unsigned row = (unsigned)xk_clampw(i, ny, pery) * (unsigned)nx;
    const unsigned rowm = (unsigned)xk_clampw(i - 1, ny, pery) * (unsigned)nx;
    const unsigned rowp = (unsigned)xk_clampw(i + 1, ny, pery) * (unsigned)nx;
    const int p2 = !pery && i == 0 && B.ky0 == BC_WALL ? 3 : 1;
    const int p4 = !pery && i == ny - 1 && B.ky1 == BC_WALL ? 1 : 3;
    const unsigned o1 = (row + xm) * (unsigned)sizeof(T), o2 = (rowm + xw) * (unsigned)sizeof(T);
    const unsigned o3 = (row + xp) * (unsigned)sizeof(T), o4 = (rowp + xw) * (unsigned)sizeof(T);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        f[4 * c + 0] = xk_at(src + (4 * c + 0) * ps, o1);
        f[4 * c + 1] = xk_at(src + (4 * c + p2) * ps, o2);
        f[4 * c + 2] = xk_at(src + (4 * c + 2) * ps, o3);
        f[4 * c + 3] = xk_at(src + (4 * c + p4) * ps, o4);
    }
}

// Vector buffer store of one value; the hardware drops it when the byte offset
// is at or beyond the resource's size (non-output lanes add kXkDrop), so stores
// need no branch.  aux 2: non-temporal.
constexpr unsigned kXkDrop = 0x80000000u;
__device__ __forceinline__ void xk_store(__amdgpu_buffer_rsrc_t r, unsigned off, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(
        __builtin_bit_cast(__attribute__((ext_vector_type(2))) int, v), r, off, 0,
        kXkNtF64 ? 2 : 0);
}
__device__ __forceinline__ void xk_store(__amdgpu_buffer_rsrc_t r, unsigned off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_int(v), r, off, 0, kXkNtF32 ? 2 : 0);
}

// Intermediate levels whose e1 / e3 exchange goes through LDS.
template <typename T, int K>
constexpr int xk_lds_levels()
{
    constexpr int L = sizeof(T) == 8 ? kXkLdsLevelsF64 : kXkLdsLevelsF32;
    return K >= kXkLdsMinK ? (L < K - 1 ? L : K - 1) : 0;
}
// Elements per LDS row of an exchange level (wide strips: two edge slots).
constexpr int xk_lds_width(int sw) { return sw > 1 ? 66 : 64; }
// Intermediate levels exchanged through LDS rows on wide strips, at most:
// FP64 6 (with 66-element rows, 4 wavefronts take 76 KiB and two workgroups
// share a compute unit), FP32 7.
constexpr int kXkWideLdsF64 = 6;
constexpr int kXkWideLdsF32 = 7;
template <typename T, int K, int SW>
constexpr int xk_lds_levels_sw()
{
    constexpr int cap = sizeof(T) == 8 ? kXkWideLdsF64 : kXkWideLdsF32;
    return SW > 1 ? (K - 1 < cap ? K - 1 : cap) : xk_lds_levels<T, K>();
}
// Wide strips: edge slots per wavefront of the register levels, and its junk area.
template <typename T, int K, int SW>
constexpr int xk_edge_slots()
{
    return (K - 1 - xk_lds_levels_sw<T, K, SW>()) * 6 * 2;
}
// LDS elements per wavefront on wide strips: the exchange-level rows, the edge
// slots of the register levels, and the junk area (as large as the slots plus
// one element per lane and parity).
template <typename T, int K, int SW>
constexpr int xk_wide_rows()
{
    return xk_lds_levels_sw<T, K, SW>() * 6 * xk_lds_width(SW) + 2 * xk_edge_slots<T, K, SW>() +
           66;
}
// LDS elements per wavefront (at least one, so the array is never empty).
template <typename T, int K>
constexpr int xk_lds_elems()
{
    return xk_lds_levels<T, K>() > 0 ? xk_lds_levels<T, K>() * 6 * 64 : 1;
}

// Grids with non-periodic faces: intermediate levels whose e1 / e3 exchange goes
// through a per-wavefront LDS row (a face lane reads its own slot instead of its
// neighbour's), at most kXkbLdsLevelsF64 (FP64) / kXkbLdsLevelsF32, in
// launches of at least kXkbLdsMinK steps; the other levels exchange in
// registers (DPP).
constexpr int kXkbLdsLevelsF64 = 6;
constexpr int kXkbLdsLevelsF32 = 7;
constexpr int kXkbLdsMinK = 2;
template <typename T, int K>
constexpr int xkb_lds_levels()
{
    constexpr int L = sizeof(T) == 8 ? kXkbLdsLevelsF64 : kXkbLdsLevelsF32;
    return K >= kXkbLdsMinK ? (L < K - 1 ? L : K - 1) : 0;
}
// Elements per exchange row of the bounded kernel: one slot per lane and, for
// FP64 storage, slot 64 holding the inflow equilibrium of the row's plane at the
// x face it is read through (e1 rows: x-, e3 rows: x+), so an inflow face lane
// pulls it with its ordinary LDS read.  (With FP32 storage the inflow value is
// not a storage value; the face lane takes it by a select.)
template <typename T>
constexpr int xkb_row_width()
{
    return sizeof(T) == 8 ? 65 : 64;
}
// Per wavefront, after the exchange rows: the inflow equilibria of the y faces'
// e2 / e4 planes (doubles at table entries 6 .. 11), read where a y-face row uses
// them, so they hold no registers across the row loop.
constexpr int kXkbFaceTab = 12;
template <typename T, int K>
constexpr int xkb_lds_elems()
{
    return xkb_lds_levels<T, K>() * 6 * xkb_row_width<T>() + kXkbFaceTab * (int)(8 / sizeof(T));
}

// v with its sign bit flipped where m has it (m: 0 or 0x80000000 per lane).
__device__ __forceinline__ double xk_xsign(double v, unsigned m)
{
    return __longlong_as_double(__double_as_longlong(v) ^ ((long long)m << 32));
}
__device__ __forceinline__ float xk_xsign(float v, unsigned m)
{
    return __int_as_float(__float_as_int(v) ^ (int)m);
}

// Output columns per strip: 64 lanes minus K - 1 halo lanes per side, rounded
// down to a whole number of aligned chunks, so (on rows that start aligned)
// each strip writes whole memory segments and never shares one with another
// strip: a partially written segment would cost the DRAM a read-modify-write.
// Grids with non-periodic faces (BND) keep at least K lanes after the last output
// column: an x+ wall node takes its own e1 at level 1 from the next lane.
// SW: wavefronts per strip (64 SW lanes).
template <typename T, int K, bool BND = false, int SW = 1>
constexpr int xk_wo()
{
    constexpr int A = (sizeof(T) == 8 ? kXkAlignF64 : kXkAlignF32) / (int)sizeof(T);
    constexpr int halo = 2 * (K - 1) + (BND ? 1 : 0), a = A > 1 ? A : 1;
    return (64 * SW - halo) / a * a;
}
// Halo lanes before the first output column (>= K - 1 on both sides).
template <typename T, int K, bool BND = false, int SW = 1>
constexpr int xk_halo()
{
    return (64 * SW - xk_wo<T, K, BND, SW>()) / 2;
}

// LDS exchange levels of a wavefront.  Each level has six rows (e1 planes c,
// e3 planes 3 + c) of xk_lds_width(SW) elements; `row` is the element index of
// the wavefront's first row in the workgroup's LDS array, and the other fields
// are per-lane element offsets within a row: where the lane reads its e1 / e3
// pull (from lane l - 1 / l + 1) and writes its own e1 / e3.
//   One wavefront per strip: 64 columns, column l = lane l.
//   Wide strips: an e1 row holds two edge slots (columns 0, 1: one per row
//   parity) and lane l at column l + 2; an e3 row holds lane l at column l and
//   two edge slots (64, 65).  Lane 63 writes its e1 into the next wavefront's
//   edge slot and lane 0 its e3 into the previous one's (no lane of its own
//   wavefront reads them); lane 0 / 63 read those slots.  The slots alternate
//   with the row parity, and the workgroup meets one barrier per row, so a slot
//   is never written while its previous value may still be read.
//   Wide strips, levels exchanged in registers (cross-lane permutes): only the
//   edge values go through LDS, in slots [level][e1 (c), e3 (3 + c)][parity] of
//   each wavefront (er: read base); ew1 / ew3 point the edge lanes' stores at
//   the neighbour's slots and every other lane's at a junk area of its own, so
//   the stores need no branch.
struct XkLds {
    int row;
    int r1, r3, w1, w3;
    int er, ew1, ew3;
    int w;  // wavefront within the strip
};

// One iteration j of the row loop.  cur: level-n pulls of this iteration's
// level-1 row; nxt (the buffer consumed in the previous iteration): receives
// those of iteration j + D, whose rows' byte offsets are onext (always a row of
// the grid, also past the segment's end).  em: e2 planes of each intermediate
// level one row below the row this iteration consumes (it is overwritten with
// the newest row, the other array then holding the older one).  There is no
// branch: levels without a valid row yet (the first 2 (K - 1) iterations) and
// iterations past the end compute values that are never stored nor reach a
// stored value, and their stores, like those of non-output lanes, carry an
// offset the hardware drops -- so the compiler's memory waits see one straight
// sequence and keep the D rows of loads in flight.
// Grids with non-periodic faces (BND): s1 / s3 hold the lane's own e1 / e3
// planes of the last row, unshifted, and the exchange happens where they are
// used (DPP), so a face lane can take its own values instead; ec is the other
// e2 array (the e2 planes of the last row), i the level-1 row of this
// iteration and inext that of the row prefetched now (both unwrapped), the
// lane's columns (xm, xw, xp), bx0 / bx1 its face flags and B the face rules.
// The y faces reuse the e2 arrays: when row 0 of level k is computed, the e2
// slot of row -1 (whose only reader is row 0's pull through the y- face)
// receives the face value; on a Neumann y+ face the e2 slot of row ny - 1 (read
// only by row ny, outside the grid) receives its own e4 planes, which row
// ny - 1 pulls back.
// X: the wavefront's LDS offsets for this row (XkLds).
template <typename T, int K, bool BND, int SW = 1>
__device__ __forceinline__ void xk_row(const T *__restrict__ src, long ps, const Phys &P,
                                       int lane, const __amdgpu_buffer_rsrc_t *orsrc,
                                       unsigned ooff, const XkOff &onext, const T (&cur)[12],
                                       T (&nxt)[12], T (&em)[K - 1][3], T (&s1)[K - 1][3],
                                       T (&s3)[K - 1][3], T (&pend)[12], unsigned &pend_off,
                                       T *__restrict__ lds, const Geo &G, const XkBnd &B, int i,
                                       int inext, int xm, int xw, int xp, bool bx0, bool bx1,
                                       T (&ec)[K - 1][3], const XkLds &X)
{
    constexpr int L = BND ? 0 : xk_lds_levels_sw<T, K, SW>();
    constexpr int LB = BND ? xkb_lds_levels<T, K>() : 0;
    const double *ftab =
        reinterpret_cast<const double *>(lds + LB * 6 * xkb_row_width<T>());  // kXkbFaceTab
    // x walls on the LDS levels: the face lane's read takes its own opposite
    // plane; the normal momentum (component 1) changes sign
    const unsigned m1 = bx0 && B.kx0 == BC_WALL ? 0x80000000u : 0u;
    const unsigned m3 = bx1 && B.kx1 == BC_WALL ? 0x80000000u : 0u;
    double v[12];
#pragma unroll
    for (int pl = 0; pl < 12; ++pl) v[pl] = (double)cur[pl];
    if constexpr (BND) {
        const bool by0 = B.ky0 != BC_PERIODIC && i == 0;
        const bool by1 = B.ky1 != BC_PERIODIC && i == G.ny - 1;
        // y walls: the opposite plane was loaded; negate the normal momentum (qy)
        if (by0 && B.ky0 == BC_WALL) v[9] = -v[9];
        if (by1 && B.ky1 == BC_WALL) v[11] = -v[11];
        // x walls: the node's own e3 (x-) / e1 (x+) was loaded by the lane outside
        // the face, whose clamped e3 / e1 pull is the face node itself
        if (B.kx0 == BC_WALL) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T t = xk_shr(cur[4 * c + 2]);
                if (bx0) v[4 * c + 0] = (double)(c == 1 ? -t : t);
            }
        }
        if (B.kx1 == BC_WALL) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T t = xk_shl(cur[4 * c + 0]);
                if (bx1) v[4 * c + 2] = (double)(c == 1 ? -t : t);
            }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (bx0 && B.kx0 == BC_INFLOW) v[4 * c + 0] = B.in1[c];
            if (bx1 && B.kx1 == BC_INFLOW) v[4 * c + 2] = B.in3[c];
            if (by0 && B.ky0 == BC_INFLOW) v[4 * c + 1] = ftab[6 + c];
            if (by1 && B.ky1 == BC_INFLOW) v[4 * c + 3] = ftab[9 + c];
        }
    }
    // The previous row's outputs are stored only now, after this row's loaded
    // values have been consumed: the wait for those loads (issued D rows ago)
    // then finds no fresh stores issued after them, and the memory counter,
    // which counts stores and loads together, does not stall on this row's
    // stores.  The scheduling barrier keeps that order.
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int pl = 0; pl < 12; ++pl) xk_store(orsrc[pl], pend_off, pend[pl]);
    if constexpr (BND)
        xk_load_clamp(src, ps, G, B, inext, xm, xw, xp, nxt);
    else
        xk_load(src, ps, onext, nxt);
    // LDS exchange levels: each level's e1 / e3 pulls are read one level ahead
    // (before the previous level's arithmetic), so the LDS latency overlaps it
    constexpr int RW = BND ? xkb_row_width<T>() : xk_lds_width(SW);
    constexpr bool PF = sizeof(T) == 4 && K <= kXkLdsPrefetchF32MaxK;
    T pf1[3], pf3[3];
    if constexpr (L > 0 && PF) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            pf1[c] = lds[X.row + c * RW + X.r1];
            pf3[c] = lds[X.row + (3 + c) * RW + X.r3];
        }
    }
    collide2d<T>(v, P);  // level 1
    // Levels 2 .. K.  Grids with non-periodic y faces: the rows near them (a
    // uniform test per iteration) run a copy of the level loop with the y-face
    // rules, so the other rows carry no per-level face conditions.
    auto levels = [&](auto yc) __attribute__((always_inline)) {
        constexpr bool Y = decltype(yc)::value;
#pragma unroll
        for (int k = 1; k < K; ++k) {
            // v: level k, one row above the level-k+1 row computed here
#pragma unroll
            for (int pl = 0; pl < 12; ++pl) v[pl] = (double)(T)v[pl];
            double o[12];
            if constexpr (BND) {
                // rr: row of level k + 1 computed here; the level-k row in v is rr + 1
                const int rr = i - k;
                const bool ry1 = Y && B.ky1 != BC_PERIODIC && rr == G.ny - 1;
                const bool vy0 = Y && B.ky0 != BC_PERIODIC && rr + 1 == 0;
                // a y- inflow value reaches row 0 through the e2 slot of row -1 (vy0);
                // with FP32 storage it is not a storage value, so row 0 takes it here
                const bool ry0 = sizeof(T) == 4 && Y && B.ky0 == BC_INFLOW && rr == 0;
                const bool vn1 = Y && B.ky1 == BC_NEUMANN && rr + 1 == G.ny - 1;
                // LDS level: this wavefront's six rows of level k (e1 planes c, e3
                // planes 3 + c); X.r1 / X.r3 count from the component's e1 row and
                // point at lane l - 1's e1 / lane l + 1's e3 of the previous row, or on
                // a face lane at its own e1 / e3 (Neumann), its own opposite plane
                // (wall, whose normal momentum is negated here) or the row's inflow
                // slot (FP64)
                const bool lv = k - 1 < LB;
                T *row = lds + X.row + (k - 1) * 6 * RW;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const T uc = ec[k - 1][c];
                    double a1, a3;
                    if (lv) {
                        const T t1 = row[c * RW + X.r1], t3 = row[c * RW + X.r3];
                        a1 = (double)(c == 1 ? xk_xsign(t1, m1) : t1);
                        a3 = (double)(c == 1 ? xk_xsign(t3, m3) : t3);
                        if constexpr (sizeof(T) == 4) {
                            if (bx0 && B.kx0 == BC_INFLOW) a1 = B.in1[c];
                            if (bx1 && B.kx1 == BC_INFLOW) a3 = B.in3[c];
                        }
                    } else {
                        const T u1 = s1[k - 1][c], u3 = s3[k - 1][c];
                        a1 = (double)xk_shr(u1);
                        a3 = (double)xk_shl(u3);
                        if (bx0)
                            a1 = B.kx0 == BC_NEUMANN ? (double)u1
                                 : B.kx0 == BC_WALL  ? (double)(c == 1 ? -u3 : u3)
                                                     : B.in1[c];
                        if (bx1)
                            a3 = B.kx1 == BC_NEUMANN ? (double)u3
                                 : B.kx1 == BC_WALL  ? (double)(c == 1 ? -u1 : u1)
                                                     : B.in3[c];
                    }
                    double a2 = (double)em[k - 1][c], a4 = v[4 * c + 3];
                    if (ry0) a2 = ftab[6 + c];
                    if (ry1)
                        a4 = B.ky1 == BC_INFLOW ? ftab[9 + c]
                             : B.ky1 == BC_WALL ? (double)(c == 2 ? -uc : uc)
                                                : (double)uc;
                    o[4 * c + 0] = a1;
                    o[4 * c + 1] = a2;
                    o[4 * c + 2] = a3;
                    o[4 * c + 3] = a4;
                    const T w2 = (T)v[4 * c + 1], w4 = (T)v[4 * c + 3];
                    em[k - 1][c] = vn1 ? w4 : w2;
                    if (vy0)
                        ec[k - 1][c] = B.ky0 == BC_WALL ? (c == 2 ? -w4 : w4)
                                       : B.ky0 == BC_INFLOW && sizeof(T) == 8 ? (T)ftab[6 + c]
                                                                              : w2;
                    if (!lv) {
                        s1[k - 1][c] = (T)v[4 * c + 0];
                        s3[k - 1][c] = (T)v[4 * c + 2];
                    }
                }
                if (lv) {
                    // overwrite with this row once every lane has read the previous one
                    __asm__ __volatile__("" ::: "memory");
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        row[c * RW + X.w1] = (T)v[4 * c + 0];
                        row[(3 + c) * RW + X.w3] = (T)v[4 * c + 2];
                    }
                    __asm__ __volatile__("" ::: "memory");
                }
            } else if (k - 1 < L) {
                // this wavefront's LDS row of level k: planes e1 (c) and e3 (3 + c);
                // read the previous row's neighbours, then overwrite with this row
                // (the wavefront executes in lockstep and its LDS operations in
                // order; the compiler barriers keep the reads before the writes and
                // the writes before the next row's reads)
                // (the per-lane offsets are loop invariant and the row index a
                // constant, so each access is one address register plus an
                // immediate offset)
                T *row = lds + X.row + (k - 1) * 6 * RW;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if constexpr (!PF) {
                        pf1[c] = row[c * RW + X.r1];
                        pf3[c] = row[(3 + c) * RW + X.r3];
                    }
                    o[4 * c + 0] = (double)pf1[c];
                    o[4 * c + 1] = (double)em[k - 1][c];
                    o[4 * c + 2] = (double)pf3[c];
                    o[4 * c + 3] = v[4 * c + 3];
                    em[k - 1][c] = (T)v[4 * c + 1];
                }
                __asm__ __volatile__("" ::: "memory");
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    row[c * RW + X.w1] = (T)v[4 * c + 0];
                    row[(3 + c) * RW + X.w3] = (T)v[4 * c + 2];
                }
                __asm__ __volatile__("" ::: "memory");
                if (PF && k < L) {
                    // the next level's pulls, written one row ago
                    T *nrow = row + 6 * RW;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        pf1[c] = nrow[c * RW + X.r1];
                        pf3[c] = nrow[(3 + c) * RW + X.r3];
                    }
                }
            } else {
                const bool el = SW > 1 && lane == 0 && X.w > 0;
                const bool er = SW > 1 && lane == 63 && X.w < SW - 1;
                const int kk = (k - 1 - L) * 12;  // this level's edge slots
                if constexpr (SW > 1) __asm__ __volatile__("" ::: "memory");
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    T a1 = s1[k - 1][c], a3 = s3[k - 1][c];
                    if constexpr (SW > 1) {
                        const T t1 = lds[X.er + kk + 2 * c], t3 = lds[X.er + kk + 2 * (3 + c)];
                        a1 = el ? t1 : a1;
                        a3 = er ? t3 : a3;
                    }
                    o[4 * c + 0] = (double)a1;
                    o[4 * c + 1] = (double)em[k - 1][c];
                    o[4 * c + 2] = (double)a3;
                    o[4 * c + 3] = v[4 * c + 3];
                    em[k - 1][c] = (T)v[4 * c + 1];
                    s1[k - 1][c] = xk_xch((T)v[4 * c + 0], lane, 1);
                    s3[k - 1][c] = xk_xch((T)v[4 * c + 2], lane, -1);
                    if constexpr (SW > 1) {
                        lds[X.ew1 + kk + 2 * c] = (T)v[4 * c + 0];
                        lds[X.ew3 + kk + 2 * (3 + c)] = (T)v[4 * c + 2];
                    }
                }
                if constexpr (SW > 1) __asm__ __volatile__("" ::: "memory");
            }
            collide2d<T>(o, P);
#pragma unroll
            for (int pl = 0; pl < 12; ++pl) v[pl] = o[pl];
        }
    };
    if constexpr (BND) {
        // the levels' rows i - k (k = 1 .. K - 1) and i - k + 1 meet a face row
        const bool yface = (B.ky0 != BC_PERIODIC && i >= -1 && i <= K - 1) ||
                           (B.ky1 != BC_PERIODIC && i >= G.ny - 1 && i <= G.ny + K - 2);
        if (yface)
            levels(std::true_type{});
        else
            levels(std::false_type{});
    } else {
        levels(std::false_type{});
    }
#pragma unroll
    for (int pl = 0; pl < 12; ++pl) pend[pl] = (T)v[pl];
    pend_off = ooff;
}

constexpr int xk_gcd(int a, int b) { return b == 0 ? a : xk_gcd(b, a % b); }

// D = rows of level-n pulls in flight ahead of the row being computed (a ring of
// D + 1 register buffers); the loop is unrolled by lcm(2, D + 1) so every ring
// slot and e2 array is addressed statically, and runs a whole number of
// unrolled blocks (the extra iterations store nothing).
// One wavefront: column strip `strip` of the grid (G, P) in src / dst, output
// rows [y0, y1).
// lds: the workgroup's LDS array, rows: its elements per wavefront (the
// wavefront's part starts at w rows); with 64-lane strips, the wavefront's own
// array and rows = 0.  Wide strips (SW > 1): wavefront w of the workgroup takes
// lanes [64 w, 64 w + 64) of the strip; every wavefront of the workgroup runs
// the same rows and meets one barrier per row.
// PRIO (the single-grid launches): the wavefront lowers its issue priority as it
// passes each quarter of its rows.  A launch is one round of workgroups, and the
// issue arbiter favours the older wavefronts, so the first workgroup on a compute
// unit otherwise finishes well before the second, which then runs alone; with the
// priority falling with progress, the wavefronts behind are issued first and the
// workgroups finish closer together (4096^2: FP64 8-step launch about 2 % shorter,
// bounded 3-4 %; the batched launches, whose tiles differ in length, are not
// helped).  Issue order does not change any value.
template <typename T, int K, int D, bool BND = false, int SW = 1, bool PRIO = false>
__device__ __forceinline__ void xk_wave(const T *__restrict__ src, T *__restrict__ dst,
                                        const Geo &G, const Phys &P, int strip, int y0, int y1,
                                        T *__restrict__ lds, int rows = 0)
{
    constexpr int WO = xk_wo<T, K, BND, SW>();  // output columns per strip
    constexpr int H = xk_halo<T, K, BND, SW>();
    static_assert(H >= K - 1 && 64 * SW - H - WO >= K - 1 + (BND ? 1 : 0), "halo lanes");
    static_assert(SW == 1 || !BND, "wide strips: all-periodic grids only");
    constexpr int U = 2 * (D + 1) / xk_gcd(2, D + 1);
    const int nx = G.nx, ny = G.ny;
    const long ps = G.ps;
    const int lane = threadIdx.x & 63;
    const int wv = SW > 1 ? (int)(threadIdx.x >> 6) : 0;  // wavefront within the strip
    const int gl = 64 * wv + lane;                        // lane within the strip
    const int x0 = strip * WO;                            // first output column
    const int xc = x0 - H + gl;                           // this lane's column, unwrapped
    // LDS offsets per row parity p (XkLds)
    XkLds Lp[2];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        Lp[p].row = wv * rows;
        Lp[p].w = wv;
        Lp[p].er = Lp[p].ew1 = Lp[p].ew3 = 0;
        if constexpr (SW > 1) {
            const bool el = lane == 0 && wv > 0, er = lane == 63 && wv < SW - 1;
            Lp[p].r1 = el ? p : lane + 1;
            Lp[p].w1 = er ? rows + p : lane + 2;
            Lp[p].r3 = er ? 64 + p : lane + 1;
            Lp[p].w3 = el ? 64 + p - rows : lane;
            // edge slots of the register levels and the junk area (xk_wide_rows)
            constexpr int lr = xk_lds_levels_sw<T, K, SW>() * 6 * xk_lds_width(SW);
            constexpr int ne = xk_edge_slots<T, K, SW>();
            const int junk = wv * rows + lr + ne + lane + p;
            Lp[p].er = wv * rows + lr + p;
            Lp[p].ew1 = er ? (wv + 1) * rows + lr + p : junk;
            Lp[p].ew3 = el ? (wv - 1) * rows + lr + p : junk;
        } else {
            Lp[p].r1 = (lane - 1) & 63;
            Lp[p].w1 = lane;
            Lp[p].r3 = (lane + 1) & 63;
            Lp[p].w3 = lane;
        }
    }
    XkBnd B{};
    bool bx0 = false, bx1 = false, clampx = false;
    if constexpr (BND) {
        B = xk_bnd<T>(G, P);
        clampx = B.kx0 != BC_PERIODIC;
        bx0 = clampx && xc == 0;
        bx1 = clampx && xc == nx - 1;
        // LDS levels (xk_row): both read offsets count from the component's e1 row
        // (the e3 row is 3 rows further); a face lane reads its own slot, a wall
        // lane the opposite plane's, an inflow lane (FP64) the row's inflow slot
        constexpr int RWB = xkb_row_width<T>();
        constexpr bool slot = RWB > 64;
        const int s1 = B.kx0 == BC_WALL ? 3 * RWB + lane : slot && B.kx0 == BC_INFLOW ? 64 : lane;
        const int s3 = B.kx1 == BC_WALL ? lane
                       : slot && B.kx1 == BC_INFLOW ? 3 * RWB + 64
                                                    : 3 * RWB + lane;
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            Lp[p].r1 = bx0 ? s1 : (lane - 1) & 63;
            Lp[p].r3 = bx1 ? s3 : 3 * RWB + ((lane + 1) & 63);
        }
        if constexpr (slot) {
            // the inflow slots of every exchange row (row 6 k + q of level k + 1:
            // q < 3 e1 plane q, else e3 plane q - 3), never overwritten
            constexpr int nrows = 6 * xkb_lds_levels<T, K>();
            if (lane < nrows) {
                const int q = lane % 6;
                const double x = q == 0 ? B.in1[0] : q == 1 ? B.in1[1] : q == 2 ? B.in1[2]
                                 : q == 3 ? B.in3[0] : q == 4 ? B.in3[1] : B.in3[2];
                lds[lane * RWB + 64] = (T)x;
            }
        }
        // the y faces' inflow values go to the wavefront's LDS table (kXkbFaceTab)
        {
            double *ft = reinterpret_cast<double *>(lds + xkb_lds_levels<T, K>() * 6 *
                                                              xkb_row_width<T>());
            if (lane < 3) {
                ft[6 + lane] = lane == 0 ? B.in2[0] : lane == 1 ? B.in2[1] : B.in2[2];
                ft[9 + lane] = lane == 0 ? B.in4[0] : lane == 1 ? B.in4[1] : B.in4[2];
            }
            __asm__ __volatile__("" ::: "memory");
        }
        // a lane needs at most one x face's inflow values (x- on bx0 lanes, x+ on
        // bx1 lanes): keep that one per lane, which frees their scalar registers
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double x = bx0 ? B.in1[c] : B.in3[c];
            B.in1[c] = x;
            B.in3[c] = x;
        }
    }
    // the lane's column and its neighbours: wrapped, or clamped to the grid
    const int xw = clampx ? min(max(xc, 0), nx - 1) : ((xc % nx) + nx) % nx;
    const int xm = clampx ? min(max(xc - 1, 0), nx - 1) : (xw == 0 ? nx - 1 : xw - 1);
    const int xp = clampx ? min(max(xc + 1, 0), nx - 1) : (xw == nx - 1 ? 0 : xw + 1);
    const bool olane = gl >= H && gl < H + WO && xc < nx;
    const int niter = (y1 - y0) + 2 * (K - 1);
    // Output row of iteration j is y0 - 2 (K - 1) + j, stored when it lies in
    // [y0, y1); byte offset of (row, xc) within a plane, or a dropped offset.
    const unsigned plane_bytes = (unsigned)nx * (unsigned)ny * (unsigned)sizeof(T);
    const unsigned ostep = (unsigned)nx * (unsigned)sizeof(T);
    const unsigned lane_off = olane ? (unsigned)xc * (unsigned)sizeof(T) : kXkDrop;
    __amdgpu_buffer_rsrc_t orsrc[12];
#pragma unroll
    for (int pl = 0; pl < 12; ++pl)
        orsrc[pl] = __builtin_amdgcn_make_buffer_rsrc(dst + pl * ps, 0, (int)plane_bytes,
                                                      0x00020000);
    int rl = (((y0 - (K - 1)) % ny) + ny) % ny;  // level-1 row of the last load, wrapped
    int il = y0 - (K - 1);                       // the same, unwrapped

    // state of the intermediate levels 1 .. K-1 (index k-1), storage precision:
    // e2 planes of the last two rows (e2[0] / e2[1] alternate), e1 planes of the
    // last row from lane l-1 and e3 planes from lane l+1
    T e2[2][K - 1][3], s1[K - 1][3], s3[K - 1][3];
#pragma unroll
    for (int k = 0; k < K - 1; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            e2[0][k][c] = e2[1][k][c] = s1[k][c] = s3[k][c] = (T)0;
        }

    T buf[D + 1][12];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        if constexpr (BND)
            xk_load_clamp(src, ps, G, B, il, xm, xw, xp, buf[d]);
        else
            xk_load(src, ps, xk_offsets<T>(rl, nx, ny, xm, xw, xp), buf[d]);
        if (d + 1 < D) {
            rl = rl == ny - 1 ? 0 : rl + 1;
            ++il;
        }
    }
    T pend[12];  // outputs of the last row, stored one iteration later
    unsigned pend_off = kXkDrop;
#pragma unroll
    for (int pl = 0; pl < 12; ++pl) pend[pl] = (T)0;
    // PRIO: the row iterations in four quarters (whole unrolled blocks), the issue
    // priority set before each; otherwise one range
    constexpr int NQ = PRIO ? 4 : 1;
    const int nblk = (niter + U - 1) / U;
    for (int qt = 0; qt < NQ; ++qt) {
        if constexpr (PRIO) {
            if (qt == 0)
                __builtin_amdgcn_s_setprio(3);
            else if (qt == 1)
                __builtin_amdgcn_s_setprio(2);
            else if (qt == 2)
                __builtin_amdgcn_s_setprio(1);
            else
                __builtin_amdgcn_s_setprio(0);
        }
        const int jb = nblk * qt / NQ * U, je = nblk * (qt + 1) / NQ * U;
        for (int j = jb; j < je; j += U) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int jj = j + u;
                const int orow = y0 - 2 * (K - 1) + jj;
                // reads from the previous row's parity, writes to this row's
                const XkLds X{Lp[0].row,        Lp[(u + 1) % 2].r1, Lp[(u + 1) % 2].r3,
                              Lp[u % 2].w1,     Lp[u % 2].w3,       Lp[(u + 1) % 2].er,
                              Lp[u % 2].ew1,    Lp[u % 2].ew3,      wv};
                if constexpr (SW > 1) {
                    // every wavefront has written the previous row's edge values;
                    // this row's slots were last read one row ago
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
                    __builtin_amdgcn_s_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
                }
                const unsigned ooff = (orow >= y0 && orow < y1)
                                          ? (unsigned)orow * ostep + lane_off
                                          : kXkDrop;
                rl = rl == ny - 1 ? 0 : rl + 1;
                ++il;
                xk_row<T, K, BND, SW>(src, ps, P, lane, orsrc, ooff,
                                  xk_offsets<T>(rl, nx, ny, xm, xw, xp), buf[u % (D + 1)],
                                  buf[(u + D) % (D + 1)], e2[u % 2], s1, s3, pend, pend_off, lds, G,
                                  B, y0 - (K - 1) + jj, il, xm, xw, xp, bx0, bx1, e2[(u + 1) % 2],
                                  X);
            }
        }
    }
#pragma unroll
    for (int pl = 0; pl < 12; ++pl) xk_store(orsrc[pl], pend_off, pend[pl]);
}

// Steps per launch at most on grids with non-periodic faces.  Measured at 4096^2
// (inflow / Neumann / wall faces), two rows in flight: FP64 K = 1 .. 5 -> 26, 42,
// 64, 74, 72 GLUPS, FP32 -> 57, 70, 108, 116, 75; beyond K = 4 the kernel spills
// registers.  In an earlier form of the kernel (level-1 face loads through
// per-lane 64-bit addresses) the FP64 K = 6 and FP32 K = 8 instantiations also
// returned wrong values over whole grids on the GPU (every face set, interior
// nodes included) with no cause found in the source, so no instantiation above
// K = 4 was built.  The present form (clamped 32-bit level-1 loads, the e1 / e3
// exchange of the intermediate levels through LDS rows, the y-face rules only in
// the iterations near a y face) equals single steps bit for bit at every K = 2 ..
// 8.  Measured at 4096^2 with the faces above: FP64 K = 2 .. 8 -> 47, 67, 92, 115,
// 132, 121, 115 GLUPS (one wavefront per SIMD from K = 7), FP32 -> 73, 105, 149,
// 166, 156, 153, 155.  With the y-face rules in every iteration: FP64 90 / 109 / 85
// at K = 4 / 5 / 6, FP32 133 / 131 / 123 (K = 4 with the exchange in registers:
// 88 / 124).
constexpr int kXkMaxKBnd = 8;
// Steps per launch by default with non-periodic faces, per storage (the fastest
// at 4096^2 with the y faces' inflow values in LDS and the x faces' rules in the
// LDS reads (inflow slots, sign masks): FP64 K = 4 .. 8 92, 116, 134, 147, 119
// GLUPS, K = 7 at 241 registers and two wavefronts per SIMD, K = 8 at one (143 at
// K = 7 with the x-face selects); FP32, whose arithmetic uses fused multiply-adds,
// 148, 170, 169, 169, 171).  A copy
// of the strip loop without the x-face rules for the strips that touch no x face
// (chosen per wavefront) measured FP64 128 at K = 6 with the inflow values in
// registers (more registers in the kernel holding both copies) and FP32 185 at K =
// 8; with them in LDS, a form whose x-face strips take the y-face copy in every row
// measured FP64 127 at K = 7, FP32 152 at K = 8 (those strips set the launch time:
// the launch is one round of workgroups), so it is not used.
constexpr int kXkbDefaultKF64 = 7;
constexpr int kXkbDefaultKF32 = 8;
// Rows of level-n pulls in flight in the bounded kernel: one (at 4096^2 FP64 K = 4
// 85 GLUPS against 74 with two; the smaller ring lets two wavefronts share a SIMD).
constexpr int kXkbDepth = 1;

// ---- 1D: K steps per launch -------------------------------------------------------
// A workgroup of NT threads (1024 in the 1D launches, 256 in the persistent
// batched kernel) holds a tile of NT consecutive nodes in LDS (four planes,
// double-buffered) and advances it K steps, one node per thread, one barrier per
// step.  The tile (first node x0) starts K nodes before its NT - 2K output nodes
// [ob, ob + nout): each step invalidates one more node at each tile edge inside
// the domain, so the outputs are exact after K steps.  At a non-periodic domain
// end the face rule (Neumann / wall / inflow, as in the one-step kernel) is
// applied to the node's own previous-level values, so nothing is lost there; with
// periodic faces the tile simply wraps.  A domain with non-periodic ends that fits
// in one tile (x0 = ob = 0, nout = nx <= NT) loses nothing at either end, so it
// stays exact for any K.  Each level is rounded to the storage type, as a store
// and a reload would round it: K steps in one launch equal K single steps bit for
// bit.
constexpr int kK1Threads = 1024;

// Ghost value of plane pl beyond face (0: x-, 1: x+) of a non-periodic end, from
// the end node's own post-collision values (the one-step kernel's face rules).
__device__ __forceinline__ double k1_face(const Geo &G, int pl, int face, const double *own,
                                          const double *weq)
{
    switch (G.bc[face]) {
    case BC_NEUMANN:
        return own[pl];
    case BC_WALL: {
        const double v = own[pl ^ 1];
        return pl >= 2 ? -v : v;
    }
    default:  // BC_INFLOW
        return weq[face * 4 + pl];
    }
}

// One tile: output nodes [ob, ob + nout) of the grid (G, P) in src / dst, with
// the workgroup's LDS array sh (NT threads, nout <= NT - 2K).
template <typename T, int NT>
__device__ __forceinline__ void k1_tile(const T *__restrict__ src, T *__restrict__ dst,
                                        const Geo &G, const Phys &P, int K, int x0, int ob,
                                        int nout, T (*sh)[4][NT])
{
    const int t = threadIdx.x;
    const int nx = G.nx;
    const long ps = G.ps;
    const bool per = G.bc[0] == BC_PERIODIC;  // the two 1D faces are periodic together
    const int oe = min(ob + nout, nx);         // output nodes [ob, oe)
    const int x = x0 + t;                      // this thread's node, unwrapped
    const bool in = per || (x >= 0 && x < nx);
    const int xw = per ? ((x % nx) + nx) % nx : x;
    const int tl = t > 0 ? t - 1 : t;          // clamped neighbours (edge values are
    const int tr = t < NT - 1 ? t + 1 : t;  // invalid anyway)
    double weq[8];
#pragma unroll
    for (int face = 0; face < 2; ++face)
        if (G.bc[face] == BC_INFLOW) feq1d<T>(G.win[face][0], G.win[face][1], P, weq + 4 * face);
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (in) {
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) v[pl] = ld(src + pl * ps + xw);
    }
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) sh[0][pl][t] = (T)v[pl];
    __syncthreads();
    int b = 0;
    for (int k = 0; k < K; ++k) {
        double f[4];
        // f+ and g+ from x - 1, f- and g- from x + 1
        if (!per && x == 0) {
            f[0] = k1_face(G, 0, 0, v, weq);
            f[2] = k1_face(G, 2, 0, v, weq);
        } else {
            f[0] = (double)sh[b][0][tl];
            f[2] = (double)sh[b][2][tl];
        }
        if (!per && x == nx - 1) {
            f[1] = k1_face(G, 1, 1, v, weq);
            f[3] = k1_face(G, 3, 1, v, weq);
        } else {
            f[1] = (double)sh[b][1][tr];
            f[3] = (double)sh[b][3][tr];
        }
        collide1d<T>(f, P);
        b ^= 1;
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) {
            v[pl] = (double)(T)f[pl];
            sh[b][pl][t] = (T)v[pl];
        }
        __syncthreads();
    }
    if (in && x >= ob && x < oe) {
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) sth<2>(dst + pl * ps + xw, v[pl]);
    }
}

} // namespace lbm
