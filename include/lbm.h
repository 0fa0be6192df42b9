/*
 * lbm.h -- C ABI of liblbm.so, the MI355X (gfx950) hot path of the vectorial
 * lattice Boltzmann scheme for the shallow-water equations of F. Dubois,
 * "Simulation of strong nonlinear waves with vectorial lattice Boltzmann
 * schemes" (Sec. 1-3), in its a = 0 form: one D1Q2 (1D) or D2Q4 (2D) particle
 * set per conserved component (h, qx = h u, qy = h v).
 *
 * What one time step computes (Sec. 1 eq. 1-hyp-N-vconserv, Sec. 2
 * eq. 2-relaxation, Sec. 3):
 *   W^k = sum_j f_j^k per node; f^eq from the kinetic decomposition of the dual
 *   entropy, closed form at a = 0 with c = 1/(2 lambda):
 *     1D: f_+- = h/2 +- q c,        g_+- = q/2 +- (q^2/h + p) c
 *     2D: f_{1,3} = h/4 +- qx c,    f_{2,4} = h/4 +- qy c,
 *         gx_{1,3} = qx/4 +- Fxx c, gx_{2,4} = qx/4 +- Fxy c,
 *         gy_{1,3} = qy/4 +- Fxy c, gy_{2,4} = qy/4 +- Fyy c,
 *     p = (g/2) h^2, Fxx = qx^2/h + p, Fxy = qx qy/h, Fyy = qy^2/h + p;
 *   relaxation (BGK, one rate s on every non-conserved moment)
 *     f* = f + s (f^eq - f);
 *   streaming one cell per step along e_j (lambda = dx/dt, Sec. 2), walls by
 *   bounce-back / anti-bounce-back (Sec. 3, last paragraph).
 *
 * Conventions
 *   - Device memory for states, fields and adjoints is allocated and owned by
 *     the caller; the library only borrows pointers and never frees them.  The
 *     library owns its host context and a few small device scratch buffers
 *     (reduction partials, flags), freed by lbm_destroy / lbm_batch_destroy.
 *   - Every call is ordered on the caller's HIP stream (lbm_params.stream;
 *     NULL = the default stream).  Calls that return host values synchronise
 *     that stream.
 *   - State layout (one buffer): n_planes SoA planes, plane p at element offset
 *     p * plane_stride, each plane row-major [y][x] with row stride nx.
 *     2D planes: (h: e1..e4, qx: e1..e4, qy: e1..e4), e1 = +x, e2 = +y,
 *     e3 = -x, e4 = -y (Sec. 3 eq. 3-stencil-d2q5).  1D planes: (h: +, -;
 *     q: +, -).  D2Q5Q4Q4 / D1Q3Q2 put the rest population h_0 first:
 *     (h: 0, e1..e4, qx: e1..e4, qy: e1..e4) and (h: 0, +, -; q: +, -).  Elements are double (LBM_F64) or float (LBM_F32);
 *     arithmetic is always double.  plane_stride >= nx*ny (padding breaks
 *     power-of-two plane strides); query it with lbm_layout.
 *   - State at level n = the post-collision distribution f*(n).  Level 0 is the
 *     collision of the equilibrium of the initial fields.  Moments of the state
 *     are the conserved fields W(n).
 *   - Return codes: LBM_OK (0), LBM_WARN_SUBCHAR (> 0, non-fatal), or a
 *     negative error; lbm_last_error() gives a thread-local message.  No
 *     exception crosses the ABI.  Asynchronous device faults surface as
 *     LBM_EDEVICE at the next synchronising call.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;
typedef struct lbm_batch lbm_batch;

enum lbm_status {
    LBM_OK = 0,
    LBM_WARN_SUBCHAR = 1, /* lambda below the monotonicity bound of the lattice:
                             max(|u| + sqrt(g h)) (1D), 2 max(|u| + sqrt(g h)) (2D) */
    LBM_EINVAL = -1,      /* bad argument (null pointer, size, rate, depth, BC) */
    LBM_EDEVICE = -2,     /* HIP runtime error */
    LBM_ESTATE = -3,      /* call out of order (e.g. step before init) */
    LBM_EDIVERGED = -4    /* a check found h <= 0 or a non-finite value */
};

/* LBM_D1Q2x2 / LBM_D2Q4x3: the hot path (rest weight a = 0, BGK).
 * LBM_D1Q3Q2 / LBM_D2Q5Q4Q4: the paper's schemes with a rest population f_0 of
 * weight a >= 0 (Sec. 2 eq. 2-potentiels-st-venant-1d, Sec. 3) and moment-space
 * relaxation with one rate per non-conserved moment (eq. 2-relaxation, MRT). */
enum lbm_lattice { LBM_D1Q2x2 = 1, LBM_D2Q4x3 = 2, LBM_D1Q3Q2 = 3, LBM_D2Q5Q4Q4 = 4 };
enum lbm_storage { LBM_F64 = 64, LBM_F32 = 32 };
enum lbm_bc {
    LBM_BC_PERIODIC = 0, /* wrap around (both faces of an axis must be periodic) */
    LBM_BC_NEUMANN = 1,  /* zero-gradient ghost: the node's own post-collision value */
    LBM_BC_WALL = 2,     /* mirror ghost: bounce-back for h and the tangential
                            momentum, anti-bounce-back for the normal momentum */
    LBM_BC_INFLOW = 3    /* ghost held at f^eq of the face's inflow state */
};

typedef struct {
    int lattice;          /* lbm_lattice */
    int storage;          /* lbm_storage */
    int nx, ny;           /* nodes; ny = 1 in 1D; nx, ny >= 2 in 2D, nx >= 2 in 1D */
    double lambda;        /* lattice velocity dx/dt > 0 */
    double s;             /* relaxation rate in (0, 2) */
    double g;             /* gravity > 0, p = (g/2) h^2 */
    double a;             /* rest weight (D1Q3Q2 / D2Q5Q4Q4 only; must be 0 otherwise) */
    double rates[10];     /* D1Q3Q2 / D2Q5Q4Q4 relaxation rates of the non-conserved
                             moments, each in (0, 2); 0 entries take s.
                             1D: (J_rho, eps_rho, J_q); 2D: (J_x, J_y, eps, XX_rho,
                             f_xx, f_xy, XX_u, f_yx, f_yy, XX_v) (Sec. 2, Sec. 3) */
    int bc[4];            /* lbm_bc of faces x-, x+, y-, y+ (y faces ignored in 1D) */
    double inflow[4][3];  /* (h, qx, qy) of LBM_BC_INFLOW faces, h > 0 */
    int check_every;      /* 0 = off; else lbm_step checks the state every that
                             many steps and returns LBM_EDIVERGED on failure */
    int block;            /* threads per workgroup: 64, 128, 256 (default), 512 */
    int nodes_per_thread; /* 1 (default), 2 or 4 nodes per thread along x */
    long plane_pad;       /* extra elements between planes; < 0 = library default */
    int mem_hints;        /* bit 0: non-temporal loads, bit 1: non-temporal stores,
                             bit 2: plain workgroup order (no XCD-aware tile remap);
                             < 0 = library default */
    int fuse_steps;       /* steps per launch (temporal blocking; bitwise identical
                             to single steps): 0 = library default, else 1 .. 1024.
                             2D all-periodic grids fuse at most 8 (larger values
                             take 8; default 8 -- FP32: 6 unless the 8-step
                             launch has three workgroups per resident slot,
                             e.g. below 3072^2 -- when that launch fills at least
                             a third of the device, e.g. 1024^2 and larger, else
                             2 when the LDS
                             two-step launch has >= 1024 workgroups, else 1;
                             planes of 2 GiB or more take 1); 2D grids with
                             Neumann, wall or inflow faces at most 8 (default 7
                             for FP64, 8 for FP32 storage, or the largest fewer
                             steps whose launch fills a third of the device, else
                             1; planes of 2 GiB or
                             more take 1); 1D grids at most 16 (larger values
                             take 16; default 16), except a 1D domain with
                             non-periodic ends of at most 1024 nodes (one LDS
                             tile, nothing lost at its ends), which takes any up
                             to 1024 (default 1024).  D2Q5Q4Q4 (rest
                             population, MRT) on all-periodic grids at most 6
                             (default 5 when that launch fills a third of the
                             device, else 1), with faces 1; D1Q3Q2 as the 1D
                             grids above.  lbm_launch_info reports the choice. */
    void *f_a, *f_b;      /* caller-owned device state buffers (ping-pong) */
    void *stream;         /* hipStream_t; NULL = default stream */
    int adjoint_storage;  /* element type of adjoint buffers: 0 = the state's,
                             LBM_F64, or LBM_F32 (only with LBM_F32 states).  A
                             float state with LBM_F64 keeps lambda in double. */
} lbm_params;

/* Size of one state buffer for the given parameters (only lattice, storage, nx,
 * ny and plane_pad are read).  Outputs may be NULL.  LBM_EINVAL on bad sizes. */
int lbm_layout(const lbm_params *p, long *plane_stride, int *n_planes, size_t *bytes);

/* Validate p, create a context and write the level-0 state into p->f_a:
 * f*(0) = C(f^eq(W0)), the post-collision state of the equilibrium of the
 * initial conserved fields (Sec. 2: f^eq from the kinetic potentials; Sec. 3 for
 * 2D).  h0, qx0, qy0: device double arrays of nx*ny values row-major [y][x]
 * (qx0 / qy0 may be NULL for zero; qy0 ignored in 1D).
 * Synchronises the stream once to check min h0 > 0 (else LBM_EINVAL) and the
 * monotonicity bound (LBM_WARN_SUBCHAR, context still created). */
int lbm_init(const lbm_params *p, const double *h0, const double *qx0, const double *qy0,
             lbm_ctx **out);

/* Advance nsteps fused pull-stream + collide steps (ping-pong between f_a and
 * f_b): the transport along the lattice velocities then the relaxation of Sec. 2
 * eq. 2-relaxation (Sec. 3 for the D2Q4 vectorial scheme), with the face rules of
 * the Sec. 3 boundary paragraph.  Launches as lbm_launch_plan lists them; the
 * state does not depend on the plan.  Stream-ordered; with check_every > 0 it
 * synchronises at each check. */
int lbm_step(lbm_ctx *ctx, long nsteps);

/* One step from src into dst (both caller-owned buffers in the context's
 * layout; must not alias).  Does not touch the context's own buffers. */
int lbm_step_buffers(lbm_ctx *ctx, const void *src, void *dst);

/* Pointer to the buffer holding the current level and the number of steps done. */
int lbm_current(lbm_ctx *ctx, void **state, long *steps_done);

/* Launch plan chosen at init (any output may be NULL): steps per launch
 * (temporal blocking depth, see fuse_steps); rows per workgroup (LDS two-step
 * kernel) or per wavefront (wave-strip K-step kernel, and the D2Q5Q4Q4 K-step
 * kernel) segment, 0 for one-step and 1D launches; and, for those K-step
 * kernels, the workgroups resident on the device at once, which the segment
 * length was chosen against (0 otherwise). */
int lbm_launch_info(lbm_ctx *ctx, int *steps_per_launch, int *segment_rows,
                    long *resident_blocks);

/* The launches lbm_step(ctx, nsteps) issues from the context's current step
 * count, in order (each advances the steps of the scheme of Sec. 2 eq.
 * 2-relaxation some number of times; the state after any plan is bitwise the
 * same): ks[i] = steps of launch i, for i < min(launches, cap); *n_launches =
 * the number of launches (may be NULL).  Launches inside captured chunks are
 * listed one by one.  Launches of steps_per_launch steps, except that on 2D grids
 * a remainder of two or more steps is spread over the last launches so their
 * step counts differ by at most one (20 steps at 8 per launch: 7, 7, 6), and a
 * remainder of one step is one one-step launch.  No device work.  LBM_EINVAL for
 * nsteps < 0, cap < 0, or cap > 0 with ks NULL. */
int lbm_launch_plan(lbm_ctx *ctx, long nsteps, int *ks, int cap, long *n_launches);

/* Copy the current state to dst / overwrite it from src (device, same layout). */
int lbm_export(lbm_ctx *ctx, void *dst);
int lbm_import(lbm_ctx *ctx, const void *src);

/* Conserved fields of a state (W^k = sum_j f_j^k, eq. 1-hyp-N-vconserv) into
 * device double arrays h, qx, qy (nx*ny each, any may be NULL; qy ignored in
 * 1D).  state = NULL means the current state.  totals_host (may be NULL)
 * receives (sum h, sum qx, sum qy) in double, by a deterministic two-stage
 * reduction; that synchronises the stream. */
int lbm_moments(lbm_ctx *ctx, const void *state, double *h, double *qx, double *qy,
                double *totals_host);

/* Discrete adjoint of one step (D1Q2x2 and D2Q4x3, every face rule): the
 * transpose of the Jacobian of one step of the scheme (Sec. 2 / Sec. 3
 * equilibria at a = 0, relaxation of eq. 2-relaxation with all rates equal, then
 * streaming with the face rules).  With C the collision, S the pull-stream and
 * u^{n+1} = C(S(u^n)):
 *   v = S(f_n); mu = (d f^eq / d W (W(v)))^T lam_np1 per node;
 *   vt = (1 - s) lam_np1 + s mu (mu broadcast over each component's planes);
 *   lam_n = S^T vt: vt_j(x) goes where the pull of plane j at x read -- the
 *     upstream node x - e_j (across a periodic face: wrapped), across a Neumann
 *     face the node's own plane j, across a wall its own opposite plane with the
 *     momentum normal to the face negated, across an inflow face nowhere;
 *   dLds_partials[b] += sum over block b of lam_np1 . (f^eq(W(v)) - v).
 * f_n: a caller buffer in the state layout and storage type; lam_np1, lam_n:
 * caller buffers in the state layout whose elements are of the context's
 * adjoint storage (lbm_params.adjoint_storage; lam_n must not alias the
 * others).  dLds_partials: device double array of lbm_adjoint_partials(ctx)
 * entries, accumulated in double (zero it before the first step).  Enqueues one
 * kernel, plus one per Neumann face.  LBM_EINVAL for the rest-population
 * lattices. */
int lbm_adjoint_step(lbm_ctx *ctx, const void *f_n, const void *lam_np1, void *lam_n,
                     double *dLds_partials);
long lbm_adjoint_partials(lbm_ctx *ctx);

/* Backward sweep over one checkpoint segment in one call (the contexts of
 * lbm_adjoint_step),
 * for checkpointed gradients: from the state ck at level n0 (a caller buffer
 * in the state layout), recompute levels n0 + 1 .. n0 + nsteps - 1 by single
 * steps into work (nsteps - 1 consecutive state buffers of lbm_layout bytes
 * each; may be NULL when nsteps == 1), then apply nsteps adjoint steps
 * (lbm_adjoint_step) from lam^{n0 + nsteps}, held in lam_a, down to lam^{n0},
 * alternating between lam_a and lam_b (adjoint storage, not aliasing ck or
 * work).  *lam_out receives 0 when lam^{n0} ends in lam_a (nsteps even), 1 when
 * in lam_b.  Only enqueues kernels on the context's stream.  LBM_EINVAL for
 * nsteps < 1, null buffers or the contexts lbm_adjoint_step rejects. */
int lbm_adjoint_segment(lbm_ctx *ctx, const void *ck, int nsteps, void *work, void *lam_a,
                        void *lam_b, double *dLds_partials, int *lam_out);

/* Every level of a run kept, for gradients without recomputation when they fit
 * in device memory: nsteps single steps (lbm_step_buffers; the scheme of Sec. 2
 * eq. 2-relaxation) from the state `from`, writing level i into slot i - 1 of
 * levels (nsteps consecutive state buffers of lbm_layout bytes each), i = 1 ..
 * nsteps.  Does not touch the context's own buffers or step count.  Only
 * enqueues kernels.  LBM_EINVAL for nsteps < 0, null buffers, or `from`
 * overlapping levels. */
int lbm_step_levels(lbm_ctx *ctx, const void *from, int nsteps, void *levels);

/* Backward sweep over stored levels (the transposed steps of lbm_adjoint_step,
 * Sec. 2 eq. 2-relaxation): levels holds the forward states of levels n0 .. n0 +
 * nsteps - 1 in nsteps consecutive state buffers (as lbm_step_levels writes
 * them); applies nsteps adjoint steps from lam^{n0 + nsteps}, held in lam_a, down
 * to lam^{n0}, alternating between lam_a and lam_b (adjoint storage, neither
 * inside levels); *lam_out as for lbm_adjoint_segment.  Only enqueues kernels.
 * LBM_EINVAL for nsteps < 1, null buffers, aliasing, or the contexts
 * lbm_adjoint_step rejects. */
int lbm_adjoint_levels(lbm_ctx *ctx, const void *levels, int nsteps, void *lam_a, void *lam_b,
                       double *dLds_partials, int *lam_out);

/* Terminal adjoint for a loss of the final height: lam_T = dL/dh broadcast to
 * the h planes (2D four, 1D two), zero on the momentum planes (adjoint
 * storage).  dLdh: device doubles, nx*ny. */
int lbm_adjoint_terminal(lbm_ctx *ctx, const double *dLdh, void *lam_T);

/* Gradient with respect to the initial fields: (dL/dh0, dL/dqx0, dL/dqy0) =
 * J(W0)^T lam0 per node, J = d f^eq / d W (the Sec. 2 / Sec. 3 equilibria at
 * a = 0; in 1D qx is q and qy is unused); lam0 in adjoint storage.  Outputs may
 * be NULL. */
int lbm_adjoint_grad_w0(lbm_ctx *ctx, const void *lam0, const double *h0, const double *qx0,
                        const double *qy0, double *grad_h0, double *grad_qx0, double *grad_qy0);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): lbm_moments without a
 * context and without any allocation.  p describes the state's layout (lattice,
 * storage, nx, ny, plane_pad are read) and the stream (p->stream); state is a
 * device buffer in that layout.  h, qx, qy (device doubles, nx*ny, any may be
 * NULL) receive the conserved fields; totals_dev (device, 3 doubles, may be
 * NULL) receives (sum h, sum qx, sum qy) by the same kernels and summation order
 * as lbm_moments' totals, so the values are bitwise equal to them.  Nothing is
 * allocated, nothing synchronises and no memset is issued: the call only
 * enqueues kernels on p->stream, so it can be captured in a HIP graph.  The
 * per-block partial sums use a fixed device array of the library (3 MiB per
 * GPU, held until the process ends): LBM_EINVAL when totals_dev is given and
 * nx*ny exceeds 33 554 432 nodes.  Calls that overlap on one GPU (concurrent
 * streams or threads) share that array and race; order them on one stream. */
int lbm_moments_noalloc(const lbm_params *p, const void *state, double *h, double *qx,
                        double *qy, double *totals_dev);

/* Discrete microscopic entropy H(f) = sum_x sum_j h_j(f_j(x)) (Sec. 1), h_j the
 * Legendre dual of the Perthame-Bouchut potential of population j at a = 0
 * (Sec. 2 eq. 2-potentiels-st-venant-1d-suite, Sec. 3 eqs. 3-st-venant-
 * contraintes-2 / 3-st-venant-enplus), taken where the potential is convex.
 * At equilibrium sum_j h_j(f^eq_j(W)) is the macroscopic entropy
 * h |u|^2 / 2 + g h^2 / 2, and the domain is the subcharacteristic condition.
 * state = NULL means the current state.  h_node (device doubles, nx*ny, may be
 * NULL) receives the per-node sums, +inf at a node with a population outside
 * the domain.  total_host / invalid_host (may be NULL) receive the total in
 * double by a deterministic two-stage reduction (+inf if any node is) and the
 * number of populations outside the domain; asking for either synchronises
 * the stream.  LBM_EINVAL for the rest-population lattices. */
int lbm_entropy(lbm_ctx *ctx, const void *state, double *h_node, double *total_host,
                long *invalid_host);

/* Deterministic sum of n device doubles into *out_host (synchronises). */
int lbm_sum(lbm_ctx *ctx, const double *partials, long n, double *out_host);

/* Release the context (NULL-safe; never frees caller memory). */
void lbm_destroy(lbm_ctx *ctx);

/* ---- batched form: many independent problems in one persistent launch ---- */

typedef struct {
    int lattice;          /* lbm_lattice */
    int nx, ny;           /* ny = 1 in 1D */
    double lambda, s, g;
    int bc[4];            /* as lbm_params.bc */
    double inflow[4][3];
    long state_offset;    /* set by lbm_batch_layout: element offset of the
                             instance's planes inside each batch buffer */
    long node_offset;     /* set by lbm_batch_layout: offset of the instance's
                             nodes in packed field arrays (h0, moments) */
} lbm_instance;

typedef struct {
    int block;            /* threads per workgroup (64..512, multiple of 64) */
    int tile_nodes;       /* dataflow mode: target nodes per work tile (>= block) */
    int grid;             /* persistent modes: workgroups; 0 = fill the device */
    int pass_nodes;       /* dataflow mode: nodes per thread per pass, 1 or 2 (0 = 1) */
    int mode;             /* 0: dataflow -- tiles advance when their neighbours have
                                finished the previous step (no grid barrier; cannot
                                deadlock whatever the grid);
                             1: step-synchronous -- units of `block` nodes, claimed
                                by the workgroups in order, 8 to a work item; a step
                                closes when all its items are complete (any grid,
                                resident or not; bounded waits, see lbm_batch_check);
                             2: flat -- one ordinary launch per step over all instances,
                                one workgroup per unit of `block` nodes; the launch
                                boundary is the step barrier; chunks of 32 steps replay
                                a captured HIP graph.  tile_nodes, grid and pass_nodes
                                are ignored;
                             3: fused -- fuse_steps steps per launch over all
                                instances (temporal blocking, bitwise identical to
                                single steps): the 2D instances as tiles of the
                                wave-strip multi-step kernels (with any 2D
                                instance that has Neumann, wall or inflow faces,
                                by default 7 (FP64) / 8 (FP32) steps per launch
                                for the whole batch),
                                the 1D instances as
                                1024-node tiles of the 1D multi-step kernel; graph
                                chunks as in mode 2; steps that do not fill a launch
                                run as flat single steps.  block, tile_nodes, grid
                                and pass_nodes are ignored;
                             4: persistent fused -- the tiles of mode 3 (1D tiles of
                                256 nodes) in ONE launch for all the steps of a run:
                                fuse_steps steps per pass; the workgroups claim the
                                tiles of a pass in order and a pass closes when all
                                are complete (256-thread workgroups, by default as
                                many as the occupancy query reports resident; `grid`
                                caps it; bounded waits, see lbm_batch_check); steps
                                that do not fill a pass run as flat single steps
                                after it.  Bitwise identical to modes 2 and 3.
                                block, tile_nodes and pass_nodes are ignored. */
    int fuse_steps;       /* modes 3, 4: steps per launch / pass, 2 .. 8 (0 = 8, or
                             with non-periodic 2D faces 7 (FP64) / 8 (FP32); 1 is
                             rejected) */
    int direct;           /* 0: replay captured HIP graphs (default); 1: launch every
                             kernel directly on the stream (e.g. under a profiler
                             that cannot follow graph replays) */
} lbm_batch_tuning;

/* Assign state_offset / node_offset to n instances (in place) for the given
 * storage; *bytes receives the size of one batch state buffer and *nodes the
 * total node count. */
int lbm_batch_layout(lbm_instance *inst, int n, int storage, size_t *bytes, long *nodes);

/* Create a batch over caller-owned buffers f_a, f_b (lbm_batch_layout sizes).
 * tuning may be NULL (defaults).  The instances are copied. */
int lbm_batch_create(const lbm_instance *inst, int n, int storage, void *f_a, void *f_b,
                     void *stream, const lbm_batch_tuning *tuning, lbm_batch **out);

/* Level-0 state of every instance from packed device double fields (node_offset). */
int lbm_batch_init(lbm_batch *b, const double *h0, const double *qx0, const double *qy0);

/* Advance every instance by nsteps in the mode chosen at creation (tuning.mode):
 * dataflow, step-synchronous, persistent fused -- ONE persistent kernel launch
 * (replayed from a captured HIP graph; persistent fused: plus single steps for a
 * remainder below fuse_steps); flat -- one launch per step (graph chunks of 32
 * steps); fused -- one launch pair (2D, 1D) per fuse_steps steps (graph chunks).
 * Stream-ordered; lbm_batch_check reports whether a persistent launch completed. */
int lbm_batch_run(lbm_batch *b, long nsteps);

/* Synchronise the stream and report whether the last run completed: the
 * persistent kernel bounds every dependency wait and, past that bound, stops
 * all workgroups and flags the run (then LBM_EDEVICE; the state is invalid). */
int lbm_batch_check(lbm_batch *b);

/* Packed conserved fields of every instance (device doubles, may be NULL). */
int lbm_batch_moments(lbm_batch *b, double *h, double *qx, double *qy);

/* Current state buffer of the batch. */
int lbm_batch_current(lbm_batch *b, void **state, long *steps_done);

/* Number of work tiles (dataflow, fused, persistent fused) or units
 * (step-synchronous, flat), and the workgroups of the persistent launch
 * (dataflow, step-synchronous, persistent fused) or of one launch (flat; fused:
 * both launches of a step group). */
int lbm_batch_info(lbm_batch *b, int *ntiles, int *grid);

void lbm_batch_destroy(lbm_batch *b);

/* Thread-local message describing the last failure (never NULL). */
const char *lbm_last_error(void);

/* Library version string. */
const char *lbm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
