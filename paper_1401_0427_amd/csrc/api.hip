// Host side of liblbm.so: argument validation, layout, ping-pong buffers,
// HIP-graph replay of step chunks, reductions and error reporting.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>

#include "lbm.h"
#include "internal.h"
#include "multistep.h"

using namespace lbm;

// ------------------------------------------------------------------ errors ----
static thread_local char g_err[512] = "no error";

static int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(LBM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
    } while (0)

extern "C" const char *lbm_last_error(void) { return g_err; }

// Used by the other translation units of the library to report an error.
int lbm_set_error(int code, const char *msg)
{
    snprintf(g_err, sizeof g_err, "%s", msg);
    return code;
}
extern "C" const char *lbm_version(void) { return "liblbm 1.0 (gfx950, D1Q2x2 / D2Q4x3)"; }

// ------------------------------------------------------------------ layout ----
static const long kAlign = 64;        // elements: planes start on 512 B / 256 B boundaries
// Defaults from measurement on MI355X (4096^2, FP64 and FP32 storage): non-temporal
// stores with plain workgroup order beat the XCD-aware order (which spreads the
// XCDs over distant rows and multiplies the open DRAM streams); padding breaks
// power-of-two plane strides at no cost.
static const long kDefaultPad = 2048;  // elements between planes
static const int kDefaultHints = 6;    // non-temporal stores, plain workgroup order

static int nplanes_of(int lattice)
{
    switch (lattice) {
    case LBM_D1Q2x2: return 4;
    case LBM_D2Q4x3: return 12;
    case LBM_D1Q3Q2: return 5;
    default: return 13;
    }
}
static int dim_of(int lattice) { return (lattice == LBM_D1Q2x2 || lattice == LBM_D1Q3Q2) ? 1 : 2; }
static bool rest_of(int lattice) { return lattice == LBM_D1Q3Q2 || lattice == LBM_D2Q5Q4Q4; }
static size_t elem_of(int storage) { return storage == LBM_F32 ? 4 : 8; }

static int layout_of(int lattice, int storage, int nx, int ny, long pad, long *ps, int *np,
                     size_t *bytes)
{
    if (lattice < LBM_D1Q2x2 || lattice > LBM_D2Q5Q4Q4)
        return fail(LBM_EINVAL, "lattice must be one of LBM_D1Q2x2, LBM_D2Q4x3, LBM_D1Q3Q2, "
                                "LBM_D2Q5Q4Q4 (got %d)", lattice);
    if (storage != LBM_F64 && storage != LBM_F32)
        return fail(LBM_EINVAL, "storage must be LBM_F64 or LBM_F32 (got %d)", storage);
    if (dim_of(lattice) == 1 && (nx < 2 || ny != 1))
        return fail(LBM_EINVAL, "1D needs nx >= 2 and ny == 1 (got %d x %d)", nx, ny);
    if (dim_of(lattice) == 2 && (nx < 2 || ny < 2))
        return fail(LBM_EINVAL, "2D needs nx, ny >= 2 (got %d x %d)", nx, ny);
    const long n = (long)nx * ny;
    if (n > (1L << 31) / 16) return fail(LBM_EINVAL, "grid too large (%ld nodes)", n);
    if (pad < 0) pad = kDefaultPad;
    const long stride = ((n + kAlign - 1) / kAlign) * kAlign + ((pad + kAlign - 1) / kAlign) * kAlign;
    if (ps) *ps = stride;
    if (np) *np = nplanes_of(lattice);
    if (bytes) *bytes = (size_t)stride * nplanes_of(lattice) * elem_of(storage);
    return LBM_OK;
}

extern "C" int lbm_layout(const lbm_params *p, long *plane_stride, int *n_planes, size_t *bytes)
{
    if (!p) return fail(LBM_EINVAL, "null params");
    return layout_of(p->lattice, p->storage, p->nx, p->ny, p->plane_pad, plane_stride, n_planes,
                     bytes);
}

static int check_bcs(int dim, const int *bc, const double (*inflow)[3])
{
    const int nface = dim == 1 ? 2 : 4;
    for (int f = 0; f < nface; ++f) {
        if (bc[f] < LBM_BC_PERIODIC || bc[f] > LBM_BC_INFLOW)
            return fail(LBM_EINVAL, "bad boundary code %d on face %d", bc[f], f);
        if ((bc[f] == LBM_BC_PERIODIC) != (bc[f ^ 1] == LBM_BC_PERIODIC))
            return fail(LBM_EINVAL, "faces %d and %d: periodic must be paired", f, f ^ 1);
        if (bc[f] == LBM_BC_INFLOW &&
            (!(inflow[f][0] > 0.0) || !isfinite(inflow[f][0]) || !isfinite(inflow[f][1]) ||
             !isfinite(inflow[f][2])))
            return fail(LBM_EINVAL, "inflow state of face %d needs finite values and h > 0", f);
    }
    return LBM_OK;
}

static int check_phys(double lambda, double s, double g)
{
    if (!(lambda > 0.0) || !isfinite(lambda)) return fail(LBM_EINVAL, "lambda must be > 0");
    if (!(s > 0.0 && s < 2.0)) return fail(LBM_EINVAL, "relaxation rate s must be in (0, 2)");
    if (!(g > 0.0) || !isfinite(g)) return fail(LBM_EINVAL, "g must be > 0");
    return LBM_OK;
}

static void fill_geo_phys(int dim, int nx, int ny, long ps, double lambda, double s, double g,
                          const int *bc, const double (*inflow)[3], Geo &G, Phys &P)
{
    G.nx = nx;
    G.ny = ny;
    G.ps = ps;
    for (int f = 0; f < 4; ++f) {
        G.bc[f] = (dim == 1 && f >= 2) ? BC_PERIODIC : bc[f];
        for (int k = 0; k < 3; ++k) G.win[f][k] = inflow[f][k];
    }
    P.c = 0.5 / lambda;
    P.s = s;
    P.hg = 0.5 * g;
    P.g = g;
}

// --------------------------------------------------------------- context ----
struct lbm_ctx {
    lbm_params p;
    int dim;
    bool rest;  // rest-population scheme (D1Q3Q2 / D2Q5Q4Q4, MRT)
    Mrt M;
    bool f32;
    bool a32;  // adjoint buffers hold floats (else doubles)
    long ps;
    int np;
    size_t bytes;
    Geo G;
    Phys P;
    Launch L;
    int fuse;  // steps per launch (at most)
    bool x2;   // 2D two-step launches take the LDS strip kernel (all-periodic grids)
    void *buf[2];
    int cur;
    long steps;
    hipStream_t st;
    // library-owned scratch
    unsigned long long *d_speed;
    int *d_flag;
    double *d_partials;  // moments partials (3 per block)
    double *d_totals;    // 3 doubles
    double *d_adj_side;  // adjoint: own contributions of Neumann face nodes (if any)
    // captured step chunks, one per starting buffer
    hipStream_t cap;
    hipGraphExec_t chunk[2];
    int chunk_len;
    int xk_seg;     // rows per segment of the wave-strip K-step launch
    long xk_slots;  // its resident workgroups on the device
    int xk_seg_k[17];  // rows per segment of a wave-strip launch of k <= fuse steps
    int rest_seg_k[kMaxFuseRest2d + 1];  // the same for the D2Q5Q4Q4 multi-step launch
    long rest_slots;                     // its resident workgroups at the full depth
};

// Steps per captured graph: the smallest multiple of twice the steps per launch that is
// at least kChunk, so a chunk holds an even number of launches (parity preserved).
static const int kChunk = 32;
// Steps per launch on the all-periodic 2D path when fuse_steps = 0: two when the
// fused launch has at least kFuseMinBlocks workgroups (about four per compute
// unit), else one -- on small grids the fused launch has too few workgroups to
// fill the chip and the one-step kernel is faster (measured at 1024^2 and on the
// 128^2 .. 1024^2 instances of the batched manifest).
static const int kFuseMinBlocks = 1024;
// 1D: steps per launch by default and at most (tiles of 1024 nodes hold the K
// levels in LDS).
static const int kDefaultFuse1d = 16;
static const int kMaxFuse1d = 16;
// 1D domains with non-periodic ends that fit one tile (step1k_whole): steps per
// launch by default and at most (nothing is lost at the tile's ends; the 1000-node
// dam break of 400 steps runs in one launch).
static const int kFuse1dWhole = 1024;
static const int kFuseSeg = 24;  // rows per workgroup segment of the LDS two-step launch
// Rows per wavefront segment of the wave-strip launch when the device cannot be
// queried (else chosen per grid at init, step2k_seg).
static const int kXkSeg = 160;
// Default steps per launch on all-periodic 2D grids (wave-strip kernel).
// FP64: 8 (GLUPS at 1024^2 / 2048^2 / 3072^2 / 4096^2 for K = 6, 7, 8: 75, 81,
// 79 / 119, 134, 136 / 136, 155, 167 / 139, 160, 176; one step at 4096^2: 29).
// FP32 (256-lane strips): 8 on grids whose 8-step launch has at least three
// workgroups per resident slot, else 6 (K = 6, 8: 77, 70 / 151, 144 / 192, 193 /
// 217, 224; one step at 4096^2: 61).
static const int kDefaultFuse2dF64 = 8;
static const int kDefaultFuse2dF32 = 8;
static const int kDefaultFuse2dF32Small = 6;
// With non-periodic faces the wave-strip kernel takes at most
// step2k_max_k_bounded() (8) steps per launch, and step2k_default_k_bounded() by
// default (FP64 7, FP32 8): at 4096^2 (inflow / Neumann / wall faces) FP64 147
// GLUPS (one step: 28), FP32 171 (one step: 59).
// Shortest segment of a wave-strip launch (the halo rows cost 2 (K - 1) per
// segment; the segment length itself is chosen per grid, step2k_seg).  Grids
// whose launch cannot fill a third of the device keep the one- or two-step
// launches by default.
static const int kXkMinSeg = 16;
// 2D all-periodic: steps per launch at most (wave-strip kernel: K = 2 .. 8)
static const int kMaxFuse2d = 8;
// D2Q5Q4Q4 on all-periodic grids: steps per launch by default (at most
// kMaxFuseRest2d); other rest-population grids take one step per launch.
// Measured at 4096^2 (GLUPS for K = 2 .. 6): FP64 36.6, 56.5, 69.3, 105.1, 102.9;
// FP32 53.8, 81.9, 102.4, 124.3, 120.6 (one step per launch: 26.9 / 57.5).
static const int kDefaultFuseRest2d = 5;

extern "C" void lbm_destroy(lbm_ctx *c)
{
    if (!c) return;
    for (int i = 0; i < 2; ++i)
        if (c->chunk[i]) (void)hipGraphExecDestroy(c->chunk[i]);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    (void)hipFree(c->d_speed);
    (void)hipFree(c->d_flag);
    (void)hipFree(c->d_partials);
    (void)hipFree(c->d_totals);
    (void)hipFree(c->d_adj_side);
    delete c;
}

extern "C" int lbm_init(const lbm_params *p, const double *h0, const double *qx0,
                        const double *qy0, lbm_ctx **out)
{
    if (!out) return fail(LBM_EINVAL, "null output pointer");
    *out = nullptr;
    if (!p) return fail(LBM_EINVAL, "null params");
    if (!h0) return fail(LBM_EINVAL, "null h0");
    if (!p->f_a || !p->f_b) return fail(LBM_EINVAL, "null state buffer");
    if (p->f_a == p->f_b) return fail(LBM_EINVAL, "f_a and f_b must be distinct buffers");
    long ps;
    int np;
    size_t bytes;
    int rc = layout_of(p->lattice, p->storage, p->nx, p->ny, p->plane_pad, &ps, &np, &bytes);
    if (rc) return rc;
    if ((rc = check_phys(p->lambda, p->s, p->g))) return rc;
    const int dim = dim_of(p->lattice);
    const bool rest = rest_of(p->lattice);
    if ((rc = check_bcs(dim, p->bc, p->inflow))) return rc;
    double rates[10];
    if (rest) {
        if (!(p->a >= 0.0) || !isfinite(p->a)) return fail(LBM_EINVAL, "rest weight a must be >= 0");
        for (int i = 0; i < 10; ++i) {
            rates[i] = p->rates[i] == 0.0 ? p->s : p->rates[i];
            if (!(rates[i] > 0.0 && rates[i] < 2.0))
                return fail(LBM_EINVAL, "relaxation rate %d must be in (0, 2)", i);
        }
    } else if (p->a != 0.0) {
        return fail(LBM_EINVAL, "a > 0 needs LBM_D1Q3Q2 or LBM_D2Q5Q4Q4");
    }
    const int block = p->block ? p->block : 256;
    if (block != 64 && block != 128 && block != 256 && block != 512)
        return fail(LBM_EINVAL, "block must be 64, 128, 256 or 512 (got %d)", block);
    const int npt = p->nodes_per_thread ? p->nodes_per_thread : 1;
    if (npt != 1 && npt != 2 && npt != 4)
        return fail(LBM_EINVAL, "nodes_per_thread must be 1, 2 or 4 (got %d)", npt);
    if (p->check_every < 0) return fail(LBM_EINVAL, "check_every must be >= 0");
    if (p->mem_hints > 7) return fail(LBM_EINVAL, "mem_hints must be < 8");
    if (p->adjoint_storage != 0 && p->adjoint_storage != LBM_F64 && p->adjoint_storage != LBM_F32)
        return fail(LBM_EINVAL, "adjoint_storage must be 0, LBM_F64 or LBM_F32 (got %d)",
                    p->adjoint_storage);
    if (p->adjoint_storage == LBM_F32 && p->storage != LBM_F32)
        return fail(LBM_EINVAL, "a float adjoint needs float state storage");
    if (p->fuse_steps < 0 || p->fuse_steps > kFuse1dWhole)
        return fail(LBM_EINVAL, "fuse_steps must be in 0 .. %d (got %d)", kFuse1dWhole,
                    p->fuse_steps);

    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(LBM_EDEVICE, "out of host memory");
    c->p = *p;
    c->dim = dim;
    c->rest = rest;
    if (rest) {
        c->M.lam = p->lambda;
        c->M.il = 1.0 / p->lambda;
        c->M.a = p->a;
        c->M.aK = p->a * (0.5 / p->g);
        c->M.g = p->g;
        c->M.hg = 0.5 * p->g;
        c->M.c = 0.5 / p->lambda;
        for (int i = 0; i < 10; ++i) c->M.rate[i] = rates[i];
    }
    c->f32 = p->storage == LBM_F32;
    c->a32 = p->adjoint_storage == 0 ? c->f32 : p->adjoint_storage == LBM_F32;
    c->ps = ps;
    c->np = np;
    c->bytes = bytes;
    fill_geo_phys(dim, p->nx, p->ny, ps, p->lambda, p->s, p->g, p->bc, p->inflow, c->G, c->P);
    c->L.block = block;
    c->L.npt = npt;
    c->L.hints = p->mem_hints < 0 ? kDefaultHints : p->mem_hints;
    {
        const bool allper = p->bc[0] == LBM_BC_PERIODIC && p->bc[1] == LBM_BC_PERIODIC &&
                            p->bc[2] == LBM_BC_PERIODIC && p->bc[3] == LBM_BC_PERIODIC;
        int want = p->fuse_steps;
        c->x2 = allper && !rest;  // two steps per launch: the LDS strip kernel (K = 2)
        c->rest_slots = 0;
        for (int k = 0; k <= kMaxFuseRest2d; ++k) c->rest_seg_k[k] = 0;
        if (rest && dim == 2 && allper) {
            // D2Q5Q4Q4: the multi-step launch at the depth asked for (at most
            // kMaxFuseRest2d), by default kDefaultFuseRest2d when its launch fills a
            // third of the device's resident workgroups, else one step per launch
            int k = want ? (want > kMaxFuseRest2d ? kMaxFuseRest2d : want) : kDefaultFuseRest2d;
            long slots = 0;
            const int seg = k >= 2 ? rest2k_seg(c->G, c->f32, k, &slots) : 0;
            if (k >= 2 && seg > 0 && (want || 3 * rest2k_blocks(c->G, k, seg) >= slots)) {
                c->fuse = k;
                c->rest_slots = slots;
                for (int kk = 2; kk <= k; ++kk) {
                    const int sk = kk == k ? seg : rest2k_seg(c->G, c->f32, kk, nullptr);
                    c->rest_seg_k[kk] = sk > 0 ? sk : seg;
                }
            } else {
                c->fuse = 1;
            }
        } else if (rest && dim == 2)
            c->fuse = 1;
        else if (dim == 1 && step1k_whole(c->G))  // D1Q2x2 and D1Q3Q2 alike
            c->fuse = want ? want : kFuse1dWhole;
        else if (dim == 1)
            c->fuse = want ? (want > kMaxFuse1d ? kMaxFuse1d : want) : kDefaultFuse1d;
        else if ((size_t)ps * (c->f32 ? 4 : 8) < ((size_t)1 << 31)) {
            const int kmax = allper ? kMaxFuse2d : step2k_max_k_bounded();
            if (want) {
                c->fuse = want > kmax ? kmax : want;
                if (c->fuse > 2 || !c->x2) {
                    c->xk_seg = step2k_seg(c->G, c->f32, c->fuse, kXkMinSeg, nullptr,
                                           &c->xk_slots);
                    if (c->xk_seg <= 0) c->xk_seg = kXkSeg;
                }
            } else {
                int kd = !allper ? step2k_default_k_bounded(c->f32)
                         : c->f32 ? kDefaultFuse2dF32 : kDefaultFuse2dF64;
                if (allper && c->f32) {
                    long s8 = 0;
                    (void)step2k_seg(c->G, true, kDefaultFuse2dF32, kXkMinSeg, nullptr, &s8);
                    if (s8 > 0 && step2k_blocks(c->G, true, kDefaultFuse2dF32, kXkMinSeg) < 3 * s8)
                        kd = kDefaultFuse2dF32Small;
                }
                bool full = false;
                long slots = 0;
                int seg = step2k_seg(c->G, c->f32, kd, kXkMinSeg, &full, &slots);
                // with non-periodic faces, a launch of fewer steps when the default
                // one cannot fill the device (smaller grids)
                while (!allper && !(seg > 0 && full) && kd > 2) {
                    --kd;
                    seg = step2k_seg(c->G, c->f32, kd, kXkMinSeg, &full, &slots);
                }
                if (seg > 0 && full) {
                    c->fuse = kd;
                    c->xk_seg = seg;
                    c->xk_slots = slots;
                } else {
                    c->fuse = c->x2 && step2x_blocks(c->G, kFuseSeg) >= kFuseMinBlocks ? 2 : 1;
                }
            }
        } else {
            c->fuse = 1;
        }
    }
    // launches of fewer steps (the plan's shorter launches) take the segment
    // length chosen for their own depth: their kernels hold fewer registers, so
    // more workgroups are resident than for the full-depth launch
    for (int k = 0; k <= 16; ++k) c->xk_seg_k[k] = 0;
    if (dim == 2 && c->xk_seg > 0)
        for (int k = 2; k <= c->fuse && k <= kMaxFuse2d; ++k) {
            if (k == 2 && c->x2) continue;
            const int sk = k == c->fuse ? c->xk_seg
                                        : step2k_seg(c->G, c->f32, k, kXkMinSeg, nullptr, nullptr);
            c->xk_seg_k[k] = sk > 0 ? sk : c->xk_seg;
        }
    c->buf[0] = p->f_a;
    c->buf[1] = p->f_b;
    c->cur = 0;
    c->steps = 0;
    c->st = (hipStream_t)p->stream;
    c->chunk_len = 2 * c->fuse * ((kChunk + 2 * c->fuse - 1) / (2 * c->fuse));

    hipError_t e;
    const int nmb = moments_blocks(c->G);
    if ((e = hipMalloc(&c->d_speed, sizeof(unsigned long long))) != hipSuccess ||
        (e = hipMalloc(&c->d_flag, 2 * sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&c->d_partials, sizeof(double) * 3 * (size_t)nmb)) != hipSuccess ||
        (e = hipMalloc(&c->d_totals, sizeof(double) * 4)) != hipSuccess) {
        lbm_destroy(c);
        return fail(LBM_EDEVICE, "hipMalloc of scratch failed: %s", hipGetErrorString(e));
    }
    bool neumann = false;
    for (int f = 0; f < (dim == 1 ? 2 : 4); ++f) neumann = neumann || c->G.bc[f] == BC_NEUMANN;
    if (neumann && !rest &&
        (e = hipMalloc(&c->d_adj_side, sizeof(double) * 12 * (size_t)adjoint_side_len(c->G))) !=
            hipSuccess) {
        lbm_destroy(c);
        return fail(LBM_EDEVICE, "hipMalloc of scratch failed: %s", hipGetErrorString(e));
    }
    unsigned long long speed_bits = 0;
    int bad = 0;
    if ((e = hipMemsetAsync(c->d_speed, 0, sizeof(unsigned long long), c->st)) != hipSuccess ||
        (e = hipMemsetAsync(c->d_flag, 0, 2 * sizeof(int), c->st)) != hipSuccess ||
        (e = (rest ? launch_init_rest(dim, c->f32, c->buf[0], h0, qx0, qy0, c->G, c->M,
                                      c->d_speed, c->d_flag, c->st)
                   : launch_init(dim, c->f32, c->buf[0], h0, qx0, qy0, c->G, c->P, c->L,
                                 c->d_speed, c->d_flag, c->st))) != hipSuccess ||
        (e = hipMemcpyAsync(&speed_bits, c->d_speed, sizeof speed_bits, hipMemcpyDeviceToHost,
                            c->st)) != hipSuccess ||
        (e = hipMemcpyAsync(&bad, c->d_flag, sizeof bad, hipMemcpyDeviceToHost, c->st)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(c->st)) != hipSuccess) {
        lbm_destroy(c);
        return fail(LBM_EDEVICE, "initialisation failed: %s", hipGetErrorString(e));
    }
    if (bad) {
        lbm_destroy(c);
        return fail(LBM_EINVAL, "initial fields need finite values and 2^-500 < h < 2^500 "
                                 "everywhere");
    }
    *out = c;
    double speed;
    memcpy(&speed, &speed_bits, sizeof speed);
    const double need = (dim == 1 ? 1.0 : 2.0) * speed;  // a = 0 bound (a > 0: indicative)
    if (p->lambda < need)
        return fail(LBM_WARN_SUBCHAR,
                    "lambda = %g is below the monotonicity bound %g of the %s lattice "
                    "(max |u| + sqrt(g h) = %g); the run may diverge",
                    p->lambda, need, dim == 1 ? "D1Q2" : "D2Q4", speed);
    return LBM_OK;
}

static hipError_t step_once(lbm_ctx *c, const void *src, void *dst, hipStream_t st)
{
    if (c->rest) return launch_step_rest(c->dim, c->f32, src, dst, c->G, c->M, st);
    return launch_step(c->dim, c->f32, src, dst, c->G, c->P, c->L, st);
}

// k steps (1 <= k <= c->fuse) in one launch: level n in src, level n+k in dst.
static hipError_t step_k(lbm_ctx *c, int k, const void *src, void *dst, hipStream_t st)
{
    if (k == 1) return step_once(c, src, dst, st);
    if (c->rest)
        return c->dim == 1
                   ? launch_step_rest1k(c->f32, src, dst, c->G, c->M, k, st)
                   : launch_step_rest2k(c->f32, src, dst, c->G, c->M, k, c->rest_seg_k[k], st);
    if (c->dim == 2) {
        if (c->x2 && k == 2)
            return launch_step2x(c->f32, src, dst, c->G, c->P, kFuseSeg, st);
        const int seg = c->xk_seg_k[k] > 0 ? c->xk_seg_k[k] : c->xk_seg > 0 ? c->xk_seg : kXkSeg;
        return launch_step2k(c->f32, src, dst, c->G, c->P, k, seg, st);
    }
    return launch_step1k(c->f32, src, dst, c->G, c->P, k, st);
}

static int check_ctx(lbm_ctx *c)
{
    if (!c) return fail(LBM_ESTATE, "null context");
    return LBM_OK;
}

static int check_state(lbm_ctx *c, long at_step)
{
    int flag = 0;
    HIP_TRY(hipMemsetAsync(c->d_flag, 0, sizeof(int), c->st));
    if (c->rest)
        HIP_TRY(launch_moments_rest(c->dim, c->f32, c->buf[c->cur], nullptr, nullptr, nullptr,
                                    nullptr, c->d_flag, c->G, c->st, nullptr));
    else
        HIP_TRY(launch_check(c->dim, c->f32, c->buf[c->cur], c->G, c->d_flag, c->st));
    HIP_TRY(hipMemcpyAsync(&flag, c->d_flag, sizeof flag, hipMemcpyDeviceToHost, c->st));
    HIP_TRY(hipStreamSynchronize(c->st));
    if (flag)
        return fail(LBM_EDIVERGED, "state diverged (h <= 0 or non-finite) at step %ld", at_step);
    return LBM_OK;
}

// Capture kChunk steps starting from buffer `from` into a graph (once).
static int ensure_chunk(lbm_ctx *c, int from)
{
    if (c->chunk[from]) return LBM_OK;
    if (!c->cap) HIP_TRY(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    int cur = from;
    hipError_t le = hipSuccess;
    // chunk_len / fuse launches of fuse steps each; an even number of them, so
    // the chunk ends on the buffer it started from
    for (int k = 0; k < c->chunk_len / c->fuse && le == hipSuccess; ++k) {
        le = step_k(c, c->fuse, c->buf[cur], c->buf[cur ^ 1], c->cap);
        cur ^= 1;
    }
    hipError_t ee = hipStreamEndCapture(c->cap, &g);
    if (le != hipSuccess || ee != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(LBM_EDEVICE, "graph capture failed: %s",
                    hipGetErrorString(le != hipSuccess ? le : ee));
    }
    hipError_t ie = hipGraphInstantiate(&c->chunk[from], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
        c->chunk[from] = nullptr;
        return fail(LBM_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(ie));
    }
    return LBM_OK;
}

// Steps of the next launch when `todo` steps remain outside the captured chunks.
// Launches of `fuse` steps, except on 2D grids a remainder of two or more steps
// is spread over the last launches so that their step counts differ by at most
// one: a 2D K-step launch takes nearly the same time for every K from 3 to 8
// (the state is read and written once), so 20 steps run as 7 + 7 + 6 rather
// than 8 + 8 + 4 (4096^2 FP64: 2.18 vs 2.29 ms).  A remainder of one step takes
// the one-step kernel, the cheapest launch.
static int next_launch_steps(const lbm_ctx *c, long todo)
{
    const long F = c->fuse;
    if (todo <= 1 || F <= 1) return (int)(todo < 1 ? todo : 1);
    const long r = todo % F;
    if (c->dim != 2 || r <= 1) return (int)(todo < F ? todo : F);
    const long launches = (todo + F - 1) / F;
    return (int)((todo + launches - 1) / launches);
}

// Whether the next chunk_len / fuse launches of a `todo`-step run are all of
// `fuse` steps (then a captured chunk can run them); todo >= chunk_len.
static bool chunk_is_full(const lbm_ctx *c, long todo)
{
    for (int i = 0; i < c->chunk_len / c->fuse; ++i, todo -= c->fuse)
        if (next_launch_steps(c, todo) != c->fuse) return false;
    return true;
}

// The launches of nsteps steps from the context's step count, in order: chunk()
// for a captured chunk of chunk_len steps, launch(k) for one launch of k steps,
// check(at) for a state check after step `at`.  Stops at the first non-zero return.
template <typename Chunk, typename Launch, typename Check>
static int walk_plan(const lbm_ctx *c, long nsteps, Chunk &&chunk, Launch &&launch,
                     Check &&check)
{
    long done = 0, steps = c->steps;
    int rc;
    while (done < nsteps) {
        long todo = nsteps - done;
        if (c->p.check_every > 0) {
            const long to_check = c->p.check_every - (steps % c->p.check_every);
            if (todo > to_check) todo = to_check;
        }
        // chunks of full launches through the captured graph, the rest launch by launch
        while (todo > 0) {
            if (todo >= c->chunk_len && chunk_is_full(c, todo)) {
                if ((rc = chunk())) return rc;
                todo -= c->chunk_len;
                done += c->chunk_len;
                steps += c->chunk_len;
                continue;
            }
            const int k = next_launch_steps(c, todo);
            if ((rc = launch(k))) return rc;
            todo -= k;
            done += k;
            steps += k;
        }
        if (c->p.check_every > 0 && steps % c->p.check_every == 0)
            if ((rc = check(steps))) return rc;
    }
    return LBM_OK;
}

extern "C" int lbm_step(lbm_ctx *c, long nsteps)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
    return walk_plan(
        c, nsteps,
        [&]() -> int {
            int r = ensure_chunk(c, c->cur);
            if (r) return r;
            HIP_TRY(hipGraphLaunch(c->chunk[c->cur], c->st));
            c->steps += c->chunk_len;  // chunk length is even: c->cur unchanged
            return LBM_OK;
        },
        [&](int k) -> int {
            HIP_TRY(step_k(c, k, c->buf[c->cur], c->buf[c->cur ^ 1], c->st));
            c->cur ^= 1;
            c->steps += k;
            return LBM_OK;
        },
        [&](long at) -> int { return check_state(c, at); });
}

extern "C" int lbm_launch_plan(lbm_ctx *c, long nsteps, int *ks, int cap, long *n_launches)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
    if (cap < 0 || (cap > 0 && !ks)) return fail(LBM_EINVAL, "ks must hold cap >= 0 entries");
    long n = 0;
    auto put = [&](int k) {
        if (n < cap) ks[n] = k;
        ++n;
    };
    rc = walk_plan(
        c, nsteps,
        [&]() -> int {
            for (int i = 0; i < c->chunk_len / c->fuse; ++i) put(c->fuse);
            return LBM_OK;
        },
        [&](int k) -> int {
            put(k);
            return LBM_OK;
        },
        [&](long) -> int { return LBM_OK; });
    if (n_launches) *n_launches = n;
    return rc;
}

extern "C" int lbm_step_buffers(lbm_ctx *c, const void *src, void *dst)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!src || !dst) return fail(LBM_EINVAL, "null buffer");
    if (src == dst) return fail(LBM_EINVAL, "src and dst must not alias");
    HIP_TRY(step_once(c, src, dst, c->st));
    return LBM_OK;
}

extern "C" int lbm_current(lbm_ctx *c, void **state, long *steps_done)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (state) *state = c->buf[c->cur];
    if (steps_done) *steps_done = c->steps;
    return LBM_OK;
}

extern "C" int lbm_launch_info(lbm_ctx *c, int *steps_per_launch, int *segment_rows,
                               long *resident_blocks)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    const bool xk = c->dim == 2 && c->fuse >= 2 && !(c->x2 && c->fuse == 2);
    if (steps_per_launch) *steps_per_launch = c->fuse;
    if (c->rest) {
        if (segment_rows) *segment_rows = c->fuse >= 2 ? c->rest_seg_k[c->fuse] : 0;
        if (resident_blocks) *resident_blocks = c->rest_slots;
        return LBM_OK;
    }
    if (segment_rows) *segment_rows = xk ? c->xk_seg : (c->fuse == 2 ? kFuseSeg : 0);
    if (resident_blocks) *resident_blocks = xk ? c->xk_slots : 0;
    return LBM_OK;
}

extern "C" int lbm_export(lbm_ctx *c, void *dst)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!dst) return fail(LBM_EINVAL, "null destination");
    HIP_TRY(hipMemcpyAsync(dst, c->buf[c->cur], c->bytes, hipMemcpyDeviceToDevice, c->st));
    return LBM_OK;
}

extern "C" int lbm_import(lbm_ctx *c, const void *src)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!src) return fail(LBM_EINVAL, "null source");
    HIP_TRY(hipMemcpyAsync(c->buf[c->cur], src, c->bytes, hipMemcpyDeviceToDevice, c->st));
    return LBM_OK;
}

extern "C" int lbm_moments(lbm_ctx *c, const void *state, double *h, double *qx, double *qy,
                           double *totals_host)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    const void *s = state ? state : c->buf[c->cur];
    int nb = 0;
    if (c->rest)
        HIP_TRY(launch_moments_rest(c->dim, c->f32, s, h, qx, qy,
                                    totals_host ? c->d_partials : nullptr, nullptr, c->G, c->st,
                                    &nb));
    else
        HIP_TRY(launch_moments(c->dim, c->f32, s, h, qx, qy,
                               totals_host ? c->d_partials : nullptr, c->G, c->st, &nb));
    if (totals_host) {
        HIP_TRY(launch_sum(c->d_partials, nb, 3, 3, c->d_totals, c->st));
        HIP_TRY(hipMemcpyAsync(totals_host, c->d_totals, 3 * sizeof(double),
                               hipMemcpyDeviceToHost, c->st));
        HIP_TRY(hipStreamSynchronize(c->st));
        if (c->dim == 1) totals_host[2] = 0.0;
    }
    return LBM_OK;
}

extern "C" int lbm_entropy(lbm_ctx *c, const void *state, double *h_node, double *total_host,
                           long *invalid_host)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (c->rest)
        return fail(LBM_EINVAL, "the entropy diagnostic is implemented for the a = 0 lattices");
    const void *s = state ? state : c->buf[c->cur];
    const bool want = total_host || invalid_host;
    int nb = 0;
    HIP_TRY(launch_entropy(c->dim, c->f32, s, c->G, c->p.lambda, c->p.g, h_node,
                           want ? c->d_partials : nullptr, c->st, &nb));
    if (want) {
        double tot[2];
        HIP_TRY(launch_sum(c->d_partials, nb, 2, 2, c->d_totals, c->st));
        HIP_TRY(hipMemcpyAsync(tot, c->d_totals, 2 * sizeof(double), hipMemcpyDeviceToHost,
                               c->st));
        HIP_TRY(hipStreamSynchronize(c->st));
        if (total_host) *total_host = tot[0];
        if (invalid_host) *invalid_host = (long)tot[1];
    }
    return LBM_OK;
}

static int check_adjoint_ctx(lbm_ctx *c)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (c->p.lattice != LBM_D2Q4x3 && c->p.lattice != LBM_D1Q2x2)
        return fail(LBM_EINVAL, "the adjoint is implemented for the D1Q2x2 and D2Q4x3 lattices "
                                "(a = 0, BGK)");
    return LBM_OK;
}

extern "C" long lbm_adjoint_partials(lbm_ctx *c) { return c ? adjoint_blocks(c->G) : 0; }

extern "C" int lbm_adjoint_step(lbm_ctx *c, const void *f_n, const void *lam_np1, void *lam_n,
                                double *dLds_partials)
{
    int rc = check_adjoint_ctx(c);
    if (rc) return rc;
    if (!f_n || !lam_np1 || !lam_n || !dLds_partials) return fail(LBM_EINVAL, "null argument");
    if (lam_n == f_n || lam_n == lam_np1)
        return fail(LBM_EINVAL, "lam_n must not alias f_n or lam_np1");
    HIP_TRY(launch_adjoint(c->dim, c->f32, c->a32, f_n, lam_np1, lam_n, dLds_partials,
                           c->d_adj_side, c->G, c->P, c->st));
    return LBM_OK;
}

// nsteps adjoint steps from lam^{n0 + nsteps} in lam_a down to lam^{n0}, level
// n0 + i of the forward state at level(i); *lam_out = 0 when lam^{n0} ends in
// lam_a, 1 when in lam_b.
template <typename Level>
static int adjoint_sweep(lbm_ctx *c, Level &&level, int nsteps, void *lam_a, void *lam_b,
                         double *dLds_partials, int *lam_out)
{
    void *hi = lam_a, *lo = lam_b;
    for (int i = nsteps - 1; i >= 0; --i) {
        HIP_TRY(launch_adjoint(c->dim, c->f32, c->a32, level(i), hi, lo, dLds_partials,
                               c->d_adj_side, c->G, c->P, c->st));
        void *t = hi;
        hi = lo;
        lo = t;
    }
    *lam_out = hi == lam_a ? 0 : 1;
    return LBM_OK;
}

extern "C" int lbm_adjoint_segment(lbm_ctx *c, const void *ck, int nsteps, void *work,
                                   void *lam_a, void *lam_b, double *dLds_partials, int *lam_out)
{
    int rc = check_adjoint_ctx(c);
    if (rc) return rc;
    if (nsteps < 1) return fail(LBM_EINVAL, "nsteps must be >= 1");
    if (!ck || !lam_a || !lam_b || !dLds_partials || !lam_out || (nsteps > 1 && !work))
        return fail(LBM_EINVAL, "null argument");
    if (lam_a == lam_b || lam_a == ck || lam_b == ck || lam_a == work || lam_b == work)
        return fail(LBM_EINVAL, "lam_a / lam_b must not alias each other, ck or work");
    // level n0 + i: ck for i = 0, else work slot i - 1
    auto level = [&](int i) -> const void * {
        return i == 0 ? ck : (const void *)((char *)work + (size_t)(i - 1) * c->bytes);
    };
    for (int i = 1; i < nsteps; ++i)
        HIP_TRY(step_once(c, level(i - 1), (void *)level(i), c->st));
    return adjoint_sweep(c, level, nsteps, lam_a, lam_b, dLds_partials, lam_out);
}

// Whether [a, a + na) and [b, b + nb) share a byte.
static bool overlaps(const void *a, size_t na, const void *b, size_t nb)
{
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + nb && y < x + na;
}

extern "C" int lbm_step_levels(lbm_ctx *c, const void *from, int nsteps, void *levels)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return LBM_OK;
    if (!from || !levels) return fail(LBM_EINVAL, "null buffer");
    if (overlaps(from, c->bytes, levels, (size_t)nsteps * c->bytes))
        return fail(LBM_EINVAL, "from must not overlap levels");
    const void *prev = from;
    for (int i = 0; i < nsteps; ++i) {
        void *dst = (char *)levels + (size_t)i * c->bytes;
        HIP_TRY(step_once(c, prev, dst, c->st));
        prev = dst;
    }
    return LBM_OK;
}

extern "C" int lbm_adjoint_levels(lbm_ctx *c, const void *levels, int nsteps, void *lam_a,
                                  void *lam_b, double *dLds_partials, int *lam_out)
{
    int rc = check_adjoint_ctx(c);
    if (rc) return rc;
    if (nsteps < 1) return fail(LBM_EINVAL, "nsteps must be >= 1");
    if (!levels || !lam_a || !lam_b || !dLds_partials || !lam_out)
        return fail(LBM_EINVAL, "null argument");
    const size_t span = (size_t)nsteps * c->bytes;
    if (lam_a == lam_b || overlaps(lam_a, c->bytes, levels, span) ||
        overlaps(lam_b, c->bytes, levels, span))
        return fail(LBM_EINVAL, "lam_a / lam_b must not alias each other or the levels");
    auto level = [&](int i) -> const void * { return (const char *)levels + (size_t)i * c->bytes; };
    return adjoint_sweep(c, level, nsteps, lam_a, lam_b, dLds_partials, lam_out);
}

extern "C" int lbm_adjoint_terminal(lbm_ctx *c, const double *dLdh, void *lam_T)
{
    int rc = check_adjoint_ctx(c);
    if (rc) return rc;
    if (!dLdh || !lam_T) return fail(LBM_EINVAL, "null argument");
    HIP_TRY(launch_adjoint_terminal(c->dim, c->a32, dLdh, lam_T, c->G, c->st));
    return LBM_OK;
}

extern "C" int lbm_adjoint_grad_w0(lbm_ctx *c, const void *lam0, const double *h0,
                                   const double *qx0, const double *qy0, double *grad_h0,
                                   double *grad_qx0, double *grad_qy0)
{
    int rc = check_adjoint_ctx(c);
    if (rc) return rc;
    if (!lam0 || !h0) return fail(LBM_EINVAL, "null argument");
    HIP_TRY(launch_adjoint_grad_w0(c->dim, c->a32, lam0, h0, qx0, qy0, grad_h0, grad_qx0,
                                   grad_qy0,
                                   c->G, c->P, c->st));
    return LBM_OK;
}

extern "C" int lbm_sum(lbm_ctx *c, const double *partials, long n, double *out_host)
{
    int rc = check_ctx(c);
    if (rc) return rc;
    if (!partials || !out_host || n < 0) return fail(LBM_EINVAL, "bad argument");
    HIP_TRY(launch_sum(partials, n, 1, 1, c->d_totals + 3, c->st));
    HIP_TRY(hipMemcpyAsync(out_host, c->d_totals + 3, sizeof(double), hipMemcpyDeviceToHost,
                           c->st));
    HIP_TRY(hipStreamSynchronize(c->st));
    return LBM_OK;
}

// ------------------------------------------------------- allocation-free totals ----
// Per-block partial sums of lbm_moments_noalloc live in this file-scope device
// array: one copy per GPU, held until the process ends.  3 partials per block
// of 256 nodes, so at most kNoAllocMaxNodes nodes.  Host code never uses the
// array's name as a device address: the address is taken once per device with
// hipGetSymbolAddress and kept in g_scratch.
static constexpr long kNoAllocDoubles = 3L << 17;  // 3 MiB
static constexpr long kNoAllocMaxNodes = kNoAllocDoubles / 3 * 256;
static __device__ __align__(256) double scratch[kNoAllocDoubles];
static constexpr int kMaxDevices = 64;
static double *g_scratch[kMaxDevices];
static std::mutex g_scratch_mu;

// Device address of this GPU's copy of `scratch` (taken on the first call on a
// device, with that device current).
static int scratch_ptr(double **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(LBM_EDEVICE, "device %d beyond the %d the library tracks", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(LBM_EDEVICE, "hipGetSymbolAddress of the totals scratch failed: %s",
                        hipGetErrorString(e));
        g_scratch[dev] = (double *)ptr;
    }
    *out = g_scratch[dev];
    return LBM_OK;
}

extern "C" int lbm_moments_noalloc(const lbm_params *p, const void *state, double *h, double *qx,
                                   double *qy, double *totals_dev)
{
    if (!p) return fail(LBM_EINVAL, "null params");
    if (!state) return fail(LBM_EINVAL, "null state");
    long ps;
    int np;
    int rc = layout_of(p->lattice, p->storage, p->nx, p->ny, p->plane_pad, &ps, &np, nullptr);
    if (rc) return rc;
    const long n = (long)p->nx * p->ny;
    if (totals_dev && n > kNoAllocMaxNodes)
        return fail(LBM_EINVAL,
                    "lbm_moments_noalloc: %ld nodes exceed the %ld its fixed scratch supports "
                    "(use lbm_moments)",
                    n, kNoAllocMaxNodes);
    const int dim = dim_of(p->lattice);
    Geo G{};
    G.nx = p->nx;
    G.ny = p->ny;
    G.ps = ps;
    const bool f32 = p->storage == LBM_F32;
    const hipStream_t st = (hipStream_t)p->stream;
    double *sp = nullptr;
    if (totals_dev && (rc = scratch_ptr(&sp))) return rc;
    int nb = 0;
    if (rest_of(p->lattice))
        HIP_TRY(launch_moments_rest(dim, f32, state, h, qx, qy, sp, nullptr, G, st, &nb));
    else
        HIP_TRY(launch_moments(dim, f32, state, h, qx, qy, sp, G, st, &nb));
    if (totals_dev) HIP_TRY(launch_sum(sp, nb, 3, 3, totals_dev, st));
    return LBM_OK;
}
