/*
 * CPU FP64 oracle for the vectorial lattice Boltzmann shallow-water scheme of
 * F. Dubois, "Simulation of strong nonlinear waves with vectorial lattice
 * Boltzmann schemes" (D1Q3Q2 in Sec. 2, D2Q5Q4Q4 in Sec. 3).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is loaded by the test-suite, by the
 * smoke check and by the benchmark's CPU-baseline leg; the GPU library never
 * links, includes or calls it and shares no code with it.
 *
 * The oracle runs the paper's scheme literally, node by node, in double
 * precision:
 *   - it carries the rest population f_0 of the paper's schemes, so a > 0 gives
 *     D1Q3Q2 / D2Q5Q4Q4 and a = 0 gives D1Q2 / D2Q4 per component exactly
 *     (f_0^eq = a K theta vanishes and f_0 stays identically zero);
 *   - state at level n = the post-collision distribution f*(n); the initial
 *     pre-collision state is the equilibrium of the initial conserved fields;
 *   - relaxation is either BGK in distribution space or the literal
 *     moment-space MRT of eq. 2-relaxation with the paper's moment bases and
 *     equilibrium moments (Sec. 2 and Sec. 3), used as a cross-check;
 *   - the discrete adjoint (exact transpose of one step, derived by hand)
 *     gives gradients of sum_x (h(T) - hhat)^2 with respect to the initial
 *     height and the relaxation rate; a complex-step copy of the forward
 *     program (same source, REAL = double _Complex) pins it.
 *
 * Readings where the paper is silent or garbled are listed in the design notes
 * of the repository: cell-centred nodes, equilibrium initial state, mirror
 * ghost walls, equilibrium inflow ghost, g = 1 unless stated, a = 0 on the hot
 * path, and the corrected equilibrium moment eps_rho^eq (factor a restored).
 *
 * Parity pins live in tests/ (conservation, lake at rest, equilibrium moments,
 * s = 1 Lax-Friedrichs, BGK = MRT, Stoker dam break, wall reflection, D4
 * symmetry, complex-step adjoint).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_NPMAX 13
enum { ORC_BC_PERIODIC = 0, ORC_BC_NEUMANN = 1, ORC_BC_WALL = 2, ORC_BC_INFLOW = 3 };

typedef struct {
    int dim;              /* 1 or 2 */
    int nx, ny;           /* ny = 1 in 1D */
    double lambda;        /* lattice velocity dx/dt */
    double s;             /* BGK relaxation rate */
    double g;             /* gravity: p = (g/2) h^2 */
    double a;             /* rest-particle weight; 0 = D1Q2 / D2Q4 per component */
    int bc[4];            /* faces x-, x+, y-, y+ */
    double inflow[4][3];  /* (h, qx, qy) of inflow faces */
    int mrt;              /* 0 = BGK, 1 = moment-space MRT with the rates below */
    double rates[10];     /* 1D: (J_rho, eps_rho, J_q); 2D: (Jx, Jy, eps, XX_rho,
                             f_xx, f_xy, XX_u, f_yx, f_yy, XX_v) */
} orc_params;

static int orc_npop(int dim) { return dim == 1 ? 5 : 13; }

/* 1D populations: 0 f0, 1 f+, 2 f-, 3 g+, 4 g-.
 * 2D populations: 0 f0, 1..4 f_j, 5..8 gx_j, 9..12 gy_j with
 * e_1 = (1,0), e_2 = (0,1), e_3 = (-1,0), e_4 = (0,-1) (eq. 3-stencil-d2q5). */
static int orc_dir2d(int p) { return p == 0 ? 0 : ((p - 1) % 4) + 1; }

static int orc_ex(int dim, int p)
{
    if (dim == 1) {
        static const int ex1[5] = {0, 1, -1, 1, -1};
        return ex1[p];
    }
    static const int exj[5] = {0, 1, 0, -1, 0};
    return exj[orc_dir2d(p)];
}

static int orc_ey(int dim, int p)
{
    if (dim == 1) return 0;
    static const int eyj[5] = {0, 0, 1, 0, -1};
    return eyj[orc_dir2d(p)];
}

static int orc_comp(int dim, int p)
{
    if (dim == 1) return p <= 2 ? 0 : 1;
    return p <= 4 ? 0 : (p <= 8 ? 1 : 2);
}

static int orc_opposite(int dim, int p)
{
    if (dim == 1) {
        static const int op1[5] = {0, 2, 1, 4, 3};
        return op1[p];
    }
    if (p == 0) return 0;
    int base = p <= 4 ? 1 : (p <= 8 ? 5 : 9);
    int j = p - base; /* 0..3 */
    return base + (j + 2) % 4;
}

/* ---- instantiate the generic core twice -------------------------------- */
#define REAL double
#define FN(name) name##_d
#include "oracle_core.inc"
#undef REAL
#undef FN

#define REAL double _Complex
#define FN(name) name##_c
#include "oracle_core.inc"
#undef REAL
#undef FN

/* Literal moment-space relaxation, eq. 2-relaxation, with the paper's moment
 * bases and equilibrium moments.
 *   1D (Sec. 2): rho = f0+f++f-, J_rho = lambda (f+ - f-),
 *        eps_rho = lambda^2 (f+ + f- - 2 f0), q = g+ + g-, J_q = lambda (g+ - g-).
 *        Equilibria: J_rho^eq = q, J_q^eq = q^2/rho + p (the physical fluxes),
 *        eps_rho^eq = lambda^2 (rho - 3 a K theta).
 *   2D (Sec. 3): rho, J_x = lambda (f1 - f3), J_y = lambda (f2 - f4),
 *        eps = f1+f2+f3+f4 - 4 f0, XX = f1 - f2 + f3 - f4, and for g_x:
 *        q_x, f_xx = lambda (gx1 - gx3), f_xy = lambda (gx2 - gx4),
 *        XX_u = gx1 - gx2 + gx3 - gx4 (g_y likewise).
 *        Equilibria (Sec. 3 table, with the factor a of eps restored):
 *        J^eq = q, eps^eq = (1 - 5a/2) rho + (5a/4)(u^2+v^2)/g, XX^eq = 0,
 *        f_xx^eq = rho u^2 + p, f_xy^eq = f_yx^eq = rho u v, f_yy^eq = rho v^2 + p. */
static void collide_mrt_node(const orc_params *P, double s_unused, const double *f, double *fs)
{
    (void)s_unused;
    const double lam = P->lambda, g = P->g, K = 0.5 / g;
    const double *r = P->rates;
    if (P->dim == 1) {
        double rho = f[0] + f[1] + f[2];
        double J = lam * (f[1] - f[2]);
        double eps = lam * lam * (f[1] + f[2] - 2.0 * f[0]);
        double q = f[3] + f[4];
        double Jq = lam * (f[3] - f[4]);
        double u = q / rho;
        double p = 0.5 * g * rho * rho;
        double theta = g * rho - 0.5 * u * u;
        double J_eq = q;
        double eps_eq = lam * lam * (rho - 3.0 * P->a * K * theta);
        double Jq_eq = q * u + p;
        J += r[0] * (J_eq - J);
        eps += r[1] * (eps_eq - eps);
        Jq += r[2] * (Jq_eq - Jq);
        /* invert the moment map */
        double f0 = (rho - eps / (lam * lam)) / 3.0;
        double S = rho - f0;
        fs[0] = f0;
        fs[1] = 0.5 * (S + J / lam);
        fs[2] = 0.5 * (S - J / lam);
        fs[3] = 0.5 * (q + Jq / lam);
        fs[4] = 0.5 * (q - Jq / lam);
        return;
    }
    double rho = f[0] + f[1] + f[2] + f[3] + f[4];
    double Jx = lam * (f[1] - f[3]);
    double Jy = lam * (f[2] - f[4]);
    double eps = f[1] + f[2] + f[3] + f[4] - 4.0 * f[0];
    double XX = f[1] - f[2] + f[3] - f[4];
    double qx = f[5] + f[6] + f[7] + f[8];
    double fxx = lam * (f[5] - f[7]);
    double fxy = lam * (f[6] - f[8]);
    double XXu = f[5] - f[6] + f[7] - f[8];
    double qy = f[9] + f[10] + f[11] + f[12];
    double fyx = lam * (f[9] - f[11]);
    double fyy = lam * (f[10] - f[12]);
    double XXv = f[9] - f[10] + f[11] - f[12];
    double u = qx / rho, v = qy / rho;
    double p = 0.5 * g * rho * rho;
    double m_eq[10] = {
        qx, qy,
        (1.0 - 2.5 * P->a) * rho + 1.25 * P->a * (u * u + v * v) / g,
        0.0,
        rho * u * u + p, rho * u * v, 0.0,
        rho * u * v, rho * v * v + p, 0.0};
    double m[10] = {Jx, Jy, eps, XX, fxx, fxy, XXu, fyx, fyy, XXv};
    for (int l = 0; l < 10; ++l) m[l] += r[l] * (m_eq[l] - m[l]);
    Jx = m[0]; Jy = m[1]; eps = m[2]; XX = m[3];
    fxx = m[4]; fxy = m[5]; XXu = m[6]; fyx = m[7]; fyy = m[8]; XXv = m[9];
    double f0 = (rho - eps) / 5.0;
    double S = rho - f0;
    double A = 0.5 * (S + XX), B = 0.5 * (S - XX);
    fs[0] = f0;
    fs[1] = 0.5 * (A + Jx / lam);
    fs[3] = 0.5 * (A - Jx / lam);
    fs[2] = 0.5 * (B + Jy / lam);
    fs[4] = 0.5 * (B - Jy / lam);
    A = 0.5 * (qx + XXu); B = 0.5 * (qx - XXu);
    fs[5] = 0.5 * (A + fxx / lam);
    fs[7] = 0.5 * (A - fxx / lam);
    fs[6] = 0.5 * (B + fxy / lam);
    fs[8] = 0.5 * (B - fxy / lam);
    A = 0.5 * (qy + XXv); B = 0.5 * (qy - XXv);
    fs[9] = 0.5 * (A + fyx / lam);
    fs[11] = 0.5 * (A - fyx / lam);
    fs[10] = 0.5 * (B + fyy / lam);
    fs[12] = 0.5 * (B - fyy / lam);
}

static void collide_node_d(const orc_params *P, double s, const double *f, double *fs)
{
    if (P->mrt)
        collide_mrt_node(P, s, f, fs);
    else
        collide_bgk_node_d(P, s, f, fs);
}

static void collide_node_c(const orc_params *P, double _Complex s, const double _Complex *f,
                           double _Complex *fs)
{
    collide_bgk_node_c(P, s, f, fs);
}

/* ---- buffers ------------------------------------------------------------ */
typedef struct {
    int np;
    long n;
    double *mem;
    double *p[ORC_NPMAX];
} orc_field;

static int field_alloc(orc_field *F, int np, long n)
{
    F->np = np;
    F->n = n;
    F->mem = (double *)malloc(sizeof(double) * (size_t)np * (size_t)n);
    if (!F->mem) return -1;
    for (int q = 0; q < ORC_NPMAX; ++q) F->p[q] = q < np ? F->mem + (long)q * n : NULL;
    return 0;
}

static void field_free(orc_field *F) { free(F->mem); F->mem = NULL; }

static int check_params(const orc_params *P)
{
    if (!P) return -1;
    if (P->dim != 1 && P->dim != 2) return -1;
    if (P->nx < 1 || P->ny < 1) return -1;
    if (P->dim == 1 && P->ny != 1) return -1;
    if (!(P->lambda > 0) || !(P->g > 0)) return -1;
    for (int face = 0; face < 4; ++face) {
        if (P->bc[face] < 0 || P->bc[face] > 3) return -1;
        if (P->dim == 1 && face >= 2) continue;
        int other = face ^ 1;
        if ((P->bc[face] == ORC_BC_PERIODIC) != (P->bc[other] == ORC_BC_PERIODIC)) return -1;
    }
    return 0;
}

static void collide_field(const orc_params *P, double s, const orc_field *f, orc_field *fs)
{
    int np = f->np;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < f->n; ++i) {
        double fl[ORC_NPMAX], fsl[ORC_NPMAX];
        for (int q = 0; q < np; ++q) fl[q] = f->p[q][i];
        collide_node_d(P, s, fl, fsl);
        for (int q = 0; q < np; ++q) fs->p[q][i] = fsl[q];
    }
}

/* ---- exported API ------------------------------------------------------- */

int orc_npop_of(int dim) { return orc_npop(dim); }

/* Host threads of the parallel loops (results do not depend on it: every node
 * is computed independently and the reductions are done in a fixed order). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_get_threads(void) { return omp_get_max_threads(); }

/* Equilibrium distribution of one state W = (h, qx, qy) (qy ignored in 1D).
 * out receives orc_npop(dim) values in the population order above. */
int orc_feq(const orc_params *P, double h, double qx, double qy, double *out)
{
    if (!P || !out) return -1;
    double W[3] = {h, qx, qy};
    feq_node_d(P, W, out);
    return 0;
}

/* Collide one node (BGK or MRT according to P->mrt). */
int orc_collide(const orc_params *P, const double *f, double *fs)
{
    if (!P || !f || !fs) return -1;
    collide_node_d(P, P->s, f, fs);
    return 0;
}

/* Run nsteps steps from the equilibrium of (h0, qx0, qy0) (qx0/qy0 may be NULL
 * for zero).  fstar_out (npop*n, population-major) receives the post-collision
 * state f*(nsteps); fpre_out, if non-NULL, the pre-collision state f(nsteps). */
int orc_run(const orc_params *P, const double *h0, const double *qx0, const double *qy0,
            long nsteps, double *fstar_out, double *fpre_out)
{
    if (check_params(P) || !h0 || !fstar_out || nsteps < 0) return -1;
    int np = orc_npop(P->dim);
    long n = (long)P->nx * P->ny;
    orc_field a, b, fs;
    if (field_alloc(&a, np, n) || field_alloc(&b, np, n) || field_alloc(&fs, np, n)) return -2;
    init_eq_d(P, h0, qx0, qy0, a.p);
    orc_field *cur = &a, *nxt = &b;
    for (long t = 0; t < nsteps; ++t) {
        step_d(P, P->s, cur->p, fs.p, nxt->p);
        orc_field *tmp = cur; cur = nxt; nxt = tmp;
    }
    if (fpre_out) memcpy(fpre_out, cur->mem, sizeof(double) * (size_t)np * (size_t)n);
    collide_field(P, P->s, cur, &fs);
    memcpy(fstar_out, fs.mem, sizeof(double) * (size_t)np * (size_t)n);
    field_free(&a); field_free(&b); field_free(&fs);
    return 0;
}

/* Advance a post-collision state by nsteps steps in place: stream, then
 * collide (the convention of a post-collision state at every level). */
int orc_advance(const orc_params *P, double *fstar, long nsteps)
{
    if (check_params(P) || !fstar || nsteps < 0) return -1;
    int np = orc_npop(P->dim);
    long n = (long)P->nx * P->ny;
    orc_field cur, pre;
    if (field_alloc(&pre, np, n)) return -2;
    cur.np = np; cur.n = n; cur.mem = fstar;
    for (int q = 0; q < ORC_NPMAX; ++q) cur.p[q] = q < np ? fstar + (long)q * n : NULL;
    for (long t = 0; t < nsteps; ++t) {
        /* stream the post-collision field, then collide: f*(t+1) = C(S(f*(t))) */
        double feq_in[4 * ORC_NPMAX];
        for (int face = 0; face < 4; ++face)
            if (P->bc[face] == ORC_BC_INFLOW) {
                double Win[3] = {P->inflow[face][0], P->inflow[face][1], P->inflow[face][2]};
                feq_node_d(P, Win, feq_in + face * ORC_NPMAX);
            }
#pragma omp parallel for schedule(static)
        for (long i = 0; i < n; ++i) {
            const int y = (int)(i / P->nx), x = (int)(i % P->nx);
            for (int q = 0; q < np; ++q)
                pre.p[q][i] = pull_d(P, cur.p, feq_in, q, x, y);
        }
        collide_field(P, P->s, &pre, &cur);
    }
    field_free(&pre);
    return 0;
}

/* Conserved fields of a distribution (population-major npop*n array). */
int orc_moments(const orc_params *P, const double *f, double *h, double *qx, double *qy)
{
    if (!P || !f) return -1;
    int np = orc_npop(P->dim);
    long n = (long)P->nx * P->ny;
    for (long i = 0; i < n; ++i) {
        double fl[ORC_NPMAX], W[3];
        for (int q = 0; q < np; ++q) fl[q] = f[(long)q * n + i];
        moments_node_d(P->dim, fl, W);
        if (h) h[i] = W[0];
        if (qx) qx[i] = W[1];
        if (qy && P->dim == 2) qy[i] = W[2];
    }
    return 0;
}

/* ---- discrete adjoint (a = 0, BGK, 1D and 2D, every face rule) -----------
 * Forward, post-collision state u: u^0 = C(f^eq(W0)), u^{n+1} = C(S(u^n)),
 * C(v) = (1-s) v + s f^eq(W(v)), S the pull-stream with the face rules of
 * pull(), loss L = sum_x (h(u^T)(x) - hhat(x))^2.  With lam^{n} = dL/du^n:
 *   v(x) = S(u^n)(x);  mu_k(x) = sum_q lam^{n+1}_q(x) d f^eq_q / d W_k (W(v(x)));
 *   vt_p(x) = (1-s) lam^{n+1}_p(x) + s mu_{comp(p)}(x);
 *   lam^n = S^T vt: every vt_p(x) is added to the slot of u^n that pull()
 *     reads for population p at x -- the upstream node x - e_p inside the
 *     domain or across a periodic face, the node's own p across a Neumann
 *     face, its own opposite population (sign flipped for the normal momentum)
 *     across a wall; across an inflow face nothing (the ghost is a constant);
 *   dL/ds += sum_x sum_p lam^{n+1}_p(x) (f^eq_p(W(v(x))) - v_p(x));
 *   dL/dW0(x) = J(W0(x))^T lam^0(x),   J = d f^eq / d W.
 * Partial derivatives of the 2D equilibrium at a = 0 (u = qx/h, v = qy/h):
 *   d/dh   : f_j 1/4;  gx: (gh - u^2) c on 1,3 (signed), -uv c on 2,4;
 *            gy: -uv c on 1,3, (gh - v^2) c on 2,4
 *   d/dqx  : f_{1,3} +-c; gx 1/4 plus 2u c (1,3), v c (2,4); gy v c (1,3)
 *   d/dqy  : f_{2,4} +-c; gy 1/4 plus u c (1,3), 2v c (2,4); gx u c (2,4)
 * with c = 1/(2 lambda) and the sign of e_j along the flux direction.  1D
 * (f_+- = h/2 +- q c, g_+- = q/2 +- (q^2/h + (g/2) h^2) c, u = q/h):
 *   d/dh : f_+- 1/2;  g_+- +-(g h - u^2) c;   d/dq : f_+- +-c;  g_+- 1/2 +- 2 u c. */
static void adj_mu_2d(const orc_params *P, const double *W, const double *lam, double *mu)
{
    const double c = 0.5 / P->lambda, g = P->g;
    double h = W[0], u = W[1] / h, v = W[2] / h;
    double L0h = lam[1] + lam[2] + lam[3] + lam[4];
    double Lxh = lam[1] - lam[3], Lyh = lam[2] - lam[4];
    double L0x = lam[5] + lam[6] + lam[7] + lam[8];
    double Lxx = lam[5] - lam[7], Lyx = lam[6] - lam[8];
    double L0y = lam[9] + lam[10] + lam[11] + lam[12];
    double Lxy = lam[9] - lam[11], Lyy = lam[10] - lam[12];
    mu[0] = 0.25 * L0h + c * (Lxx * (g * h - u * u) - Lyx * u * v - Lxy * u * v + Lyy * (g * h - v * v));
    mu[1] = c * Lxh + 0.25 * L0x + c * (2.0 * u * Lxx + v * Lyx + v * Lxy);
    mu[2] = c * Lyh + 0.25 * L0y + c * (2.0 * v * Lyy + u * Lxy + u * Lyx);
}

static void adj_mu_1d(const orc_params *P, const double *W, const double *lam, double *mu)
{
    const double c = 0.5 / P->lambda, g = P->g;
    double h = W[0], u = W[1] / h;
    double L0f = lam[1] + lam[2], L1f = lam[1] - lam[2];
    double L0g = lam[3] + lam[4], L1g = lam[3] - lam[4];
    mu[0] = 0.5 * L0f + c * (g * h - u * u) * L1g;
    mu[1] = c * L1f + 0.5 * L0g + 2.0 * u * c * L1g;
}

static void adj_mu(const orc_params *P, const double *W, const double *lam, double *mu)
{
    if (P->dim == 1)
        adj_mu_1d(P, W, lam, mu);
    else
        adj_mu_2d(P, W, lam, mu);
}

static int adj_supported(const orc_params *P)
{
    if (check_params(P)) return 0;
    return P->a == 0.0 && !P->mrt;
}

/* Transpose of pull(): add val to the slot of the field that
 * pull(P, field, ., p, x, y) reads (nothing across an inflow face). */
static void pull_transpose(const orc_params *P, double *const *lam, int p, int x, int y,
                           double val)
{
    int nx = P->nx, ny = P->ny;
    int sx = x - orc_ex(P->dim, p), sy = y - orc_ey(P->dim, p);
    int face = -1;
    if (sx < 0) face = 0;
    else if (sx >= nx) face = 1;
    else if (sy < 0) face = 2;
    else if (sy >= ny) face = 3;
    if (face < 0) {
        lam[p][(long)sy * nx + sx] += val;
        return;
    }
    switch (P->bc[face]) {
    case ORC_BC_PERIODIC:
        sx = (sx + nx) % nx;
        sy = (sy + ny) % ny;
        lam[p][(long)sy * nx + sx] += val;
        return;
    case ORC_BC_NEUMANN:
        lam[p][(long)y * nx + x] += val;
        return;
    case ORC_BC_WALL: {
        int q = orc_opposite(P->dim, p);
        int normal = (face < 2) ? 1 : 2;
        lam[q][(long)y * nx + x] += (orc_comp(P->dim, p) == normal) ? -val : val;
        return;
    }
    default: /* ORC_BC_INFLOW */
        return;
    }
}

static void inflow_feq_d(const orc_params *P, double *feq_in)
{
    for (int face = 0; face < 4; ++face)
        if (P->bc[face] == ORC_BC_INFLOW) {
            double Win[3] = {P->inflow[face][0], P->inflow[face][1], P->inflow[face][2]};
            feq_node_d(P, Win, feq_in + face * ORC_NPMAX);
        }
}

/* One adjoint step: given the forward post-collision state u^n and lam^{n+1},
 * write lam^n and add this step's contribution to *dLds (all arrays
 * population-major, npop populations: 5 in 1D, 13 in 2D; the rest population's
 * adjoint is carried for exactness but never reaches the gradients at a = 0). */
int orc_adjoint_step(const orc_params *P, const double *un, const double *lam_np1,
                     double *lam_n, double *dLds)
{
    if (!adj_supported(P) || !un || !lam_np1 || !lam_n) return -1;
    const int np = orc_npop(P->dim), nx = P->nx, ny = P->ny;
    const long n = (long)nx * ny;
    const double s = P->s;
    double feq_in[4 * ORC_NPMAX];
    inflow_feq_d(P, feq_in);
    double *U[ORC_NPMAX], *Ln[ORC_NPMAX];
    for (int q = 0; q < np; ++q) {
        U[q] = (double *)un + (long)q * n;
        Ln[q] = lam_n + (long)q * n;
    }
    double *vt = (double *)malloc(sizeof(double) * (size_t)np * (size_t)n);
    double *row_acc = (double *)calloc((size_t)ny, sizeof(double));
    if (!vt || !row_acc) {
        free(vt);
        free(row_acc);
        return -2;
    }
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        double racc = 0.0;
        for (int x = 0; x < nx; ++x) {
            long i = (long)y * nx + x;
            double v[ORC_NPMAX], lam[ORC_NPMAX], W[3], feq[ORC_NPMAX], mu[3];
            for (int q = 0; q < np; ++q) {
                v[q] = pull_d(P, U, feq_in, q, x, y);
                lam[q] = lam_np1[(long)q * n + i];
            }
            moments_node_d(P->dim, v, W);
            feq_node_d(P, W, feq);
            adj_mu(P, W, lam, mu);
            for (int q = 0; q < np; ++q) {
                racc += lam[q] * (feq[q] - v[q]);
                vt[(long)q * n + i] = (1.0 - s) * lam[q] + s * mu[orc_comp(P->dim, q)];
            }
        }
        row_acc[y] = racc;
    }
    /* lam^n = S^T vt, in node order */
    memset(lam_n, 0, sizeof(double) * (size_t)np * (size_t)n);
    for (long i = 0; i < n; ++i) {
        const int y = (int)(i / nx), x = (int)(i % nx);
        for (int q = 0; q < np; ++q) pull_transpose(P, Ln, q, x, y, vt[(long)q * n + i]);
    }
    double acc = 0.0;
    for (int y = 0; y < ny; ++y) acc += row_acc[y];
    free(row_acc);
    free(vt);
    if (dLds) *dLds += acc;
    return 0;
}

/* Directional derivative of one step u -> C(S(u)) between post-collision levels
 * along (du, ds), by complex step of the same forward code (pull and BGK
 * collision in complex arithmetic): out = Im(C_{s + i eps ds}(S(u + i eps du))) / eps.
 * Independent of the hand-derived adjoint above. */
int orc_step_cs(const orc_params *P, const double *u, const double *du, double ds, double eps,
                double *out)
{
    if (check_params(P) || P->mrt || !u || !out || !(eps > 0)) return -1;
    const int np = orc_npop(P->dim), nx = P->nx;
    const long n = (long)nx * P->ny;
    double _Complex *mem = (double _Complex *)malloc(sizeof(double _Complex) * (size_t)np * (size_t)n);
    if (!mem) return -2;
    double _Complex *U[ORC_NPMAX];
    for (int q = 0; q < np; ++q) U[q] = mem + (long)q * n;
    for (long k = 0; k < (long)np * n; ++k) mem[k] = u[k] + I * (eps * (du ? du[k] : 0.0));
    double _Complex feq_in[4 * ORC_NPMAX];
    for (int face = 0; face < 4; ++face)
        if (P->bc[face] == ORC_BC_INFLOW) {
            double _Complex Win[3] = {P->inflow[face][0], P->inflow[face][1], P->inflow[face][2]};
            feq_node_c(P, Win, feq_in + face * ORC_NPMAX);
        }
    const double _Complex s = P->s + I * (eps * ds);
    for (long i = 0; i < n; ++i) {
        const int y = (int)(i / nx), x = (int)(i % nx);
        double _Complex v[ORC_NPMAX], fs[ORC_NPMAX];
        for (int q = 0; q < np; ++q) v[q] = pull_c(P, U, feq_in, q, x, y);
        collide_node_c(P, s, v, fs);
        for (int q = 0; q < np; ++q) out[(long)q * n + i] = cimag(fs[q]) / eps;
    }
    free(mem);
    return 0;
}

/* Loss and gradients for the adjoint workload: W0 = (h0, 0, 0) (1D: (h0, 0)),
 * T steps, L = sum (h(u^T) - hhat)^2, any face rules.  Forward states are
 * checkpointed every K steps and recomputed segment by segment in the backward
 * sweep.  grad_h0 (n) and *grad_s receive dL/dh0 and dL/ds; *loss the loss. */
int orc_loss_grad(const orc_params *P, const double *h0, const double *hhat, long T, int K,
                  double *loss, double *grad_h0, double *grad_s)
{
    if (!adj_supported(P) || !h0 || !hhat || T < 0 || K < 1) return -1;
    const int np = orc_npop(P->dim);
    const long n = (long)P->nx * P->ny;
    const size_t bytes = sizeof(double) * (size_t)np * (size_t)n;
    long nck = T / K + 1;
    double *ck = (double *)malloc(bytes * (size_t)nck);
    double *seg = (double *)malloc(bytes * (size_t)(K + 1));
    double *lamA = (double *)malloc(bytes), *lamB = (double *)malloc(bytes);
    double *cur = (double *)malloc(bytes);
    if (!ck || !seg || !lamA || !lamB || !cur) {
        free(ck); free(seg); free(lamA); free(lamB); free(cur);
        return -2;
    }
    /* u^0 = C(f^eq(W0)) */
    {
        orc_field f0, fs;
        field_alloc(&f0, np, n);
        fs.np = np; fs.n = n; fs.mem = cur;
        for (int q = 0; q < ORC_NPMAX; ++q) fs.p[q] = q < np ? cur + (long)q * n : NULL;
        init_eq_d(P, h0, NULL, NULL, f0.p);
        collide_field(P, P->s, &f0, &fs);
        field_free(&f0);
    }
    memcpy(ck, cur, bytes);
    for (long t = 0; t < T; ++t) {
        orc_advance(P, cur, 1);
        if ((t + 1) % K == 0 && (t + 1) / K < nck) memcpy(ck + (size_t)((t + 1) / K) * np * n, cur, bytes);
    }
    /* terminal adjoint: dL/du^T = 2 (h - hhat) on every population of h */
    double L = 0.0;
    memset(lamA, 0, bytes);
    for (long i = 0; i < n; ++i) {
        double fl[ORC_NPMAX], W[3];
        for (int q = 0; q < np; ++q) fl[q] = cur[(long)q * n + i];
        moments_node_d(P->dim, fl, W);
        double r = W[0] - hhat[i];
        L += r * r;
        for (int q = 0; q < np; ++q)
            if (orc_comp(P->dim, q) == 0) lamA[(long)q * n + i] = 2.0 * r;
    }
    double gs = 0.0;
    double *lam_hi = lamA, *lam_lo = lamB;
    for (long seg0 = ((T - 1) / K) * K; T > 0 && seg0 >= 0; seg0 -= K) {
        long seg1 = seg0 + K < T ? seg0 + K : T; /* states seg0 .. seg1-1 needed */
        memcpy(seg, ck + (size_t)(seg0 / K) * np * n, bytes);
        for (long t = seg0 + 1; t < seg1; ++t) {
            memcpy(seg + (size_t)(t - seg0) * np * n, seg + (size_t)(t - seg0 - 1) * np * n, bytes);
            orc_advance(P, seg + (size_t)(t - seg0) * np * n, 1);
        }
        for (long t = seg1 - 1; t >= seg0; --t) {
            orc_adjoint_step(P, seg + (size_t)(t - seg0) * np * n, lam_hi, lam_lo, &gs);
            double *tmp = lam_hi; lam_hi = lam_lo; lam_lo = tmp;
        }
    }
    /* dL/dh0 = mu_h(lam^0; W0) */
    for (long i = 0; i < n; ++i) {
        double lam[ORC_NPMAX], W[3] = {h0[i], 0.0, 0.0}, mu[3];
        for (int q = 0; q < np; ++q) lam[q] = lam_hi[(long)q * n + i];
        adj_mu(P, W, lam, mu);
        if (grad_h0) grad_h0[i] = mu[0];
    }
    if (loss) *loss = L;
    if (grad_s) *grad_s = gs;
    free(ck); free(seg); free(lamA); free(lamB); free(cur);
    return 0;
}

/* The 2D name of the same function (kept for existing callers). */
int orc_loss_grad_2d(const orc_params *P, const double *h0, const double *hhat, long T, int K,
                     double *loss, double *grad_h0, double *grad_s)
{
    if (!P || P->dim != 2) return -1;
    return orc_loss_grad(P, h0, hhat, T, K, loss, grad_h0, grad_s);
}

/* Loss of the same workload evaluated in complex arithmetic at
 * (h0 + i eps dh0, s + i eps ds): the complex-step directional derivative
 * Im(L)/eps of the forward program, independent of the hand-derived adjoint.
 * 1D or 2D, any face rules; small grids only (no checkpointing). */
int orc_loss_cs_2d(const orc_params *P, const double *h0, const double *dh0, double ds,
                   const double *hhat, long T, double eps, double *loss, double *dloss)
{
    if (check_params(P) || P->mrt || !h0 || !hhat) return -1;
    const int np = orc_npop(P->dim);
    const long n = (long)P->nx * P->ny;
    double _Complex *mem = (double _Complex *)malloc(sizeof(double _Complex) * 3 * np * (size_t)n);
    double _Complex *hc = (double _Complex *)malloc(sizeof(double _Complex) * (size_t)n);
    if (!mem || !hc) { free(mem); free(hc); return -2; }
    double _Complex *A[ORC_NPMAX], *B[ORC_NPMAX], *S[ORC_NPMAX];
    for (int q = 0; q < np; ++q) {
        A[q] = mem + (long)q * n;
        B[q] = mem + (long)(np + q) * n;
        S[q] = mem + (long)(2 * np + q) * n;
    }
    for (long i = 0; i < n; ++i) hc[i] = h0[i] + I * (eps * (dh0 ? dh0[i] : 0.0));
    double _Complex s = P->s + I * (eps * ds);
    init_eq_c(P, hc, NULL, NULL, A);
    /* u^0 = C(f^eq(W0)), then u^{n+1} = C(S(u^n)); implemented as pre-collision
     * iteration f(n+1) = S(C(f(n))) followed by a final collision. */
    double _Complex **cur = A, **nxt = B;
    for (long t = 0; t < T; ++t) {
        step_c(P, s, cur, S, nxt);
        double _Complex **tmp = cur; cur = nxt; nxt = tmp;
    }
    double _Complex L = 0.0;
    for (long i = 0; i < n; ++i) {
        double _Complex fl[ORC_NPMAX], fs[ORC_NPMAX], W[3];
        for (int q = 0; q < np; ++q) fl[q] = cur[q][i];
        collide_node_c(P, s, fl, fs);
        moments_node_c(P->dim, fs, W);
        double _Complex r = W[0] - hhat[i];
        L += r * r;
    }
    if (loss) *loss = creal(L);
    if (dloss) *dloss = cimag(L) / eps;
    free(mem); free(hc);
    return 0;
}

/* ---- discrete microscopic entropy (Sec. 1, a = 0) --------------------------
 * Perthame-Bouchut potentials of the hot-path lattices, from Sec. 2 (1D,
 * eq. 2-potentiels-st-venant-1d-suite) and Sec. 3 (2D, eqs. 3-st-venant-
 * contraintes-2 and 3-st-venant-enplus) at a = 0, with phi = (theta, U) the
 * entropy variables, P = theta + |U|^2 / 2 and p = K P^2 (K = 1/(2g)):
 *   h_j^*(phi) = p(phi) (alpha + e_j . U / (2 lambda)),
 *   alpha = 1/2 (1D, e = +-1) or 1/4 (2D, e_j the four unit vectors).
 * The microscopic entropy of population j with components F = (f_j, g_j ...)
 * is the Legendre dual h_j(F) = sup_phi (phi . F - h_j^*(phi)), taken over the
 * domain where h_j^* is convex: the stationary point grad h_j^*(phi) = F is
 * found by Newton's method on the full system (Hessian of h_j^* as Jacobian),
 * started from the entropy variables of the node's conserved fields, and is
 * accepted only if the Hessian there is positive definite.  Outside that
 * domain the entropy is reported as +infinity. */
static void ent_pot(int dim, int j, double K, double lam, const double *phi, double *hs,
                    double *grad, double hess[3][3])
{
    const int n = dim == 1 ? 2 : 3;
    double e[2] = {0.0, 0.0};
    double alpha;
    if (dim == 1) {
        e[0] = j == 0 ? 1.0 : -1.0;
        alpha = 0.5;
    } else {
        static const double ex[4] = {1, 0, -1, 0}, ey[4] = {0, 1, 0, -1};
        e[0] = ex[j];
        e[1] = ey[j];
        alpha = 0.25;
    }
    const double *U = phi + 1;
    double U2 = 0.0, eU = 0.0;
    for (int a = 0; a < n - 1; ++a) {
        U2 += U[a] * U[a];
        eU += e[a] * U[a];
    }
    const double P = phi[0] + 0.5 * U2;
    const double p = K * P * P;
    const double m = alpha + eU / (2.0 * lam);
    double b[2];
    for (int a = 0; a < n - 1; ++a) b[a] = e[a] / (2.0 * lam);
    if (hs) *hs = p * m;
    if (grad) {
        grad[0] = 2.0 * K * P * m;
        for (int a = 0; a < n - 1; ++a) grad[1 + a] = 2.0 * K * P * U[a] * m + p * b[a];
    }
    if (hess) {
        hess[0][0] = 2.0 * K * m;
        for (int a = 0; a < n - 1; ++a) {
            hess[0][1 + a] = hess[1 + a][0] = 2.0 * K * U[a] * m + 2.0 * K * P * b[a];
            for (int c = 0; c < n - 1; ++c)
                hess[1 + a][1 + c] = 2.0 * K * U[a] * U[c] * m + (a == c ? 2.0 * K * P * m : 0.0) +
                                     2.0 * K * P * (U[a] * b[c] + U[c] * b[a]);
        }
    }
}

/* Solve A x = r (n <= 3) by Gaussian elimination with partial pivoting. */
static int ent_solve(int n, double A[3][3], const double *r, double *x)
{
    double M[3][4];
    for (int i = 0; i < n; ++i) {
        for (int k = 0; k < n; ++k) M[i][k] = A[i][k];
        M[i][n] = r[i];
    }
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int i = c + 1; i < n; ++i)
            if (fabs(M[i][c]) > fabs(M[piv][c])) piv = i;
        if (M[piv][c] == 0.0) return -1;
        if (piv != c)
            for (int k = 0; k <= n; ++k) {
                double t = M[c][k]; M[c][k] = M[piv][k]; M[piv][k] = t;
            }
        for (int i = c + 1; i < n; ++i) {
            double q = M[i][c] / M[c][c];
            for (int k = c; k <= n; ++k) M[i][k] -= q * M[c][k];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = M[i][n];
        for (int k = i + 1; k < n; ++k) s -= M[i][k] * x[k];
        x[i] = s / M[i][i];
    }
    return 0;
}

/* Positive definiteness by Cholesky. */
static int ent_posdef(int n, double A[3][3])
{
    double L[3][3] = {{0}};
    for (int i = 0; i < n; ++i)
        for (int k = 0; k <= i; ++k) {
            double s = A[i][k];
            for (int m = 0; m < k; ++m) s -= L[i][m] * L[k][m];
            if (i == k) {
                if (!(s > 0.0)) return 0;
                L[i][i] = sqrt(s);
            } else {
                L[i][k] = s / L[k][k];
            }
        }
    return 1;
}

/* Objective phi . F - h_j^*(phi) of the dual, and whether phi lies in the
 * convexity domain of h_j^* (Hessian positive definite). */
static int ent_obj(int dim, int j, double K, double lam, const double *F, const double *phi,
                   double *obj, double *grad, double hess[3][3])
{
    const int n = dim == 1 ? 2 : 3;
    double hs, g[3], H[3][3];
    ent_pot(dim, j, K, lam, phi, &hs, g, H);
    double dot = 0.0;
    for (int i = 0; i < n; ++i) dot += phi[i] * F[i];
    *obj = dot - hs;
    if (grad)
        for (int i = 0; i < n; ++i) grad[i] = F[i] - g[i];
    if (hess)
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < n; ++k) hess[i][k] = H[i][k];
    return ent_posdef(n, H);
}

/* Entropy of one population: j = 0 (+) / 1 (-) in 1D, 0..3 (e_1..e_4) in 2D;
 * F = its components (f, g) or (f, gx, gy).  The objective phi . F - h_j^*(phi)
 * is concave inside the convexity domain of h_j^*, so its maximiser there is
 * found by Newton ascent steps, each shortened until the new point stays in
 * the domain and the objective does not decrease.  The iteration stops when
 * the full Newton step (the distance to the maximiser to first order) is at
 * rounding level, or small and no longer shrinking (the rounding floor of a
 * nearly singular Hessian at the edge of the domain).  The start phi0 must lie
 * in the domain.  Returns 0 and writes h and phi if the maximum is attained
 * in the domain, 1 otherwise. */
static int ent_pop(int dim, int j, double K, double lam, const double *F, const double *phi0,
                   double *h_out, double *phi_out)
{
    const int n = dim == 1 ? 2 : 3;
    double phi[3] = {phi0[0], phi0[1], dim == 2 ? phi0[2] : 0.0};
    double obj, grad[3], H[3][3];
    if (!ent_obj(dim, j, K, lam, F, phi, &obj, grad, H)) return 1;
    double prev = INFINITY;
    for (int it = 0; it < 2000; ++it) {
        double d[3];
        if (ent_solve(n, H, grad, d)) return 1; /* ascent direction H^-1 (F - grad h^*) */
        double full = 0.0;
        for (int i = 0; i < n; ++i) {
            double rel = fabs(d[i]) / (1.0 + fabs(phi[i]));
            if (rel > full) full = rel;
        }
        if (!(full == full)) return 1;
        if (full <= 1e-14 || (full < 1e-10 && full >= prev)) {
            *h_out = obj;
            if (phi_out)
                for (int i = 0; i < n; ++i) phi_out[i] = phi[i];
            return 0;
        }
        prev = full;
        /* far from the maximiser the objective must not decrease; close to it
         * (full step below 1e-6, Newton's quadratic region) its change is below
         * rounding and only the domain is checked */
        const int test_obj = full >= 1e-6;
        double t = 1.0, trial[3], tobj, tgrad[3], tH[3][3];
        int accepted = 0;
        for (int k = 0; k < 80; ++k, t *= 0.5) {
            for (int i = 0; i < n; ++i) trial[i] = phi[i] + t * d[i];
            if (ent_obj(dim, j, K, lam, F, trial, &tobj, tgrad, tH) && (!test_obj || tobj >= obj)) {
                accepted = 1;
                break;
            }
        }
        if (!accepted) return 1;
        if (t < 1.0) prev = INFINITY;
        for (int i = 0; i < n; ++i) {
            phi[i] = trial[i];
            grad[i] = tgrad[i];
            for (int k = 0; k < n; ++k) H[i][k] = tH[i][k];
        }
        obj = tobj;
    }
    return 1;
}

/* A starting point inside the convexity domain of every population: U = 0 and
 * theta = 1 / (4 kappa^2) (kappa = 1/lambda in 1D, 2/lambda in 2D), where
 * h_j^* is convex (D = 1 > kappa sqrt(P) = 1/2). */
static void ent_start(int dim, double lam, double *phi)
{
    const double kappa = dim == 1 ? 1.0 / lam : 2.0 / lam;
    phi[0] = 0.25 / (kappa * kappa);
    phi[1] = 0.0;
    phi[2] = 0.0;
}

/* Entropy of one population: the ascent is started from the population's own
 * first-order point (U = (g_x, g_y) / f, P = f / (2 w K), i.e. the potential
 * read with 1 + e_j . U / (2 alpha lambda) ~ 1) when that point lies in the
 * domain, and from the generic interior point otherwise or if that fails. */
static int ent_pop_any(int dim, int j, double K, double lam, const double *F, double *h_out,
                       double *phi_out)
{
    const int n = dim == 1 ? 2 : 3;
    double phi0[3];
    if (F[0] > 0.0) {
        const double w = dim == 1 ? 0.5 : 0.25;
        double U2 = 0.0;
        for (int a = 1; a < n; ++a) {
            phi0[a] = F[a] / F[0];
            U2 += phi0[a] * phi0[a];
        }
        phi0[0] = F[0] / (2.0 * w * K) - 0.5 * U2;
        double obj, H[3][3];
        if (ent_obj(dim, j, K, lam, F, phi0, &obj, NULL, H) &&
            ent_pop(dim, j, K, lam, F, phi0, h_out, phi_out) == 0)
            return 0;
    }
    ent_start(dim, lam, phi0);
    return ent_pop(dim, j, K, lam, F, phi0, h_out, phi_out);
}

/* Entropy of one population j with components F (exported for the tests). */
int orc_entropy_pop(const orc_params *P, int j, const double *F, double *h_out, double *phi_out)
{
    if (!P || !F || !h_out || P->a != 0.0 || !(P->lambda > 0.0) || !(P->g > 0.0)) return -1;
    if (j < 0 || j >= (P->dim == 1 ? 2 : 4)) return -1;
    return ent_pop_any(P->dim, j, 0.5 / P->g, P->lambda, F, h_out, phi_out);
}

/* H(f) = sum over nodes and populations of h_j.  h_node (optional) receives
 * the per-node sums (+inf at a node with a population outside the domain),
 * *total the sum over nodes in node order (+inf if any node is), *invalid the
 * number of populations outside the domain.  a = 0 only; the rest population
 * must be zero (its potential vanishes, so its dual is finite only at 0). */
int orc_entropy(const orc_params *P, const double *f, double *h_node, double *total,
                long *invalid)
{
    if (check_params(P) || !f || P->a != 0.0) return -1;
    const int np = orc_npop(P->dim), nj = P->dim == 1 ? 2 : 4;
    const long n = (long)P->nx * P->ny;
    const double K = 0.5 / P->g;
    double tot = 0.0;
    long bad = 0;
    for (long i = 0; i < n; ++i) {
        double fl[ORC_NPMAX];
        for (int q = 0; q < np; ++q) fl[q] = f[(long)q * n + i];
        double Hn = 0.0;
        int nodebad = 0;
        if (fl[0] != 0.0) {
            ++bad;
            nodebad = 1;
        }
        for (int j = 0; j < nj; ++j) {
            double F[3], hj;
            if (P->dim == 1) {
                F[0] = fl[1 + j];
                F[1] = fl[3 + j];
            } else {
                F[0] = fl[1 + j];
                F[1] = fl[5 + j];
                F[2] = fl[9 + j];
            }
            if (ent_pop_any(P->dim, j, K, P->lambda, F, &hj, NULL)) {
                ++bad;
                nodebad = 1;
            } else {
                Hn += hj;
            }
        }
        if (nodebad) Hn = INFINITY;
        if (h_node) h_node[i] = Hn;
        tot += Hn;
    }
    if (total) *total = tot;
    if (invalid) *invalid = bad;
    return 0;
}
