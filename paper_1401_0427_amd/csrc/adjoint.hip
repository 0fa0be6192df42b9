// Discrete adjoint of the fused stream + collide step (2D and 1D, every face rule).
//
// Forward (post-collision state u):  u^{n+1} = C(S(u^n)),
//   S: pull-stream v_j(x) = u_j(x - e_j),  C(v) = (1 - s) v + s f^eq(W(v)).
// Adjoint of one step, lam^n = (dC S / du^n)^T lam^{n+1}:
//   mu_k(x)  = sum_q lam^{n+1}_q(x) d f^eq_q / d W_k at W(v(x))
//   vt_j(x)  = (1 - s) lam^{n+1}_j(x) + s mu_{k(j)}(x)
//   lam^n_j(x - e_j) = vt_j(x)              (transpose of the pull = a push)
//   dL/ds   += sum_x sum_j lam^{n+1}_j(x) (f^eq_j(W(v(x))) - v_j(x))
// With u = qx/h, v = qy/h and c = 1/(2 lambda), the partial derivatives of the
// a = 0 equilibria (Sec. 3 potentials) give
//   mu_h  = L0h/4 + c [Lxx (g h - u^2) - (Lyx + Lxy) u v + Lyy (g h - v^2)]
//   mu_qx = c Lxh + L0x/4 + c [2 u Lxx + v (Lyx + Lxy)]
//   mu_qy = c Lyh + L0y/4 + c [2 v Lyy + u (Lxy + Lyx)]
// where for each component family L0 = sum_j lam_j, L{x,y} = sum_j e_j lam_j
// (Lxx: x-moment of the gx family, Lyx: y-moment of gx, Lxy: x-moment of gy).
//
// Each workgroup adds its share of dL/ds to its own FP64 slot (no atomics), so
// the gradient is deterministic.  The adjoint may be stored in another type than
// the state (TA = double for a float state keeps lambda in double; the
// arithmetic is double throughout).
#include "internal.h"

namespace lbm {

__device__ __forceinline__ void adj_mu(const double *l, double h, double qx, double qy,
                                       const Phys &P, double &mh, double &mx, double &my)
{
    const double ih = 1.0 / h;
    const double u = qx * ih, v = qy * ih, gh = P.g * h;
    const double L0h = (l[0] + l[2]) + (l[1] + l[3]);
    const double Lxh = l[0] - l[2], Lyh = l[1] - l[3];
    const double L0x = (l[4] + l[6]) + (l[5] + l[7]);
    const double Lxx = l[4] - l[6], Lyx = l[5] - l[7];
    const double L0y = (l[8] + l[10]) + (l[9] + l[11]);
    const double Lxy = l[8] - l[10], Lyy = l[9] - l[11];
    const double cross = Lyx + Lxy;
    mh = 0.25 * L0h + P.c * (Lxx * (gh - u * u) - cross * (u * v) + Lyy * (gh - v * v));
    mx = P.c * Lxh + 0.25 * L0x + P.c * (2.0 * u * Lxx + v * cross);
    my = P.c * Lyh + 0.25 * L0y + P.c * (2.0 * v * Lyy + u * cross);
}

template <typename T, typename TA>
__global__ void __launch_bounds__(256) k_adj2d(const T *__restrict__ un,
                                               const TA *__restrict__ lam1, TA *__restrict__ lam0,
                                               double *__restrict__ partials, Geo G, Phys P,
                                               int tiles_x, int ntiles)
{
    __shared__ double sh[256];
    const int t = xcd_tile(blockIdx.x, ntiles, false);  // plain order measured faster
    const int y = t / tiles_x;
    const int x = (t - y * tiles_x) * 256 + threadIdx.x;
    const int nx = G.nx, ny = G.ny;
    const long ps = G.ps;
    double acc = 0.0;
    if (x < nx) {
        const long row = (long)y * nx;
        const int xm = x == 0 ? nx - 1 : x - 1;
        const int xp = x == nx - 1 ? 0 : x + 1;
        const long rm = y == 0 ? (long)(ny - 1) * nx : row - nx;
        const long rp = y == ny - 1 ? 0 : row + nx;
        double v[12], l[12];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const T *b = un + (4 * k) * ps;
            v[4 * k + 0] = ld(b + row + xm);
            v[4 * k + 1] = ld(b + ps + rm + x);
            v[4 * k + 2] = ld(b + 2 * ps + row + xp);
            v[4 * k + 3] = ld(b + 3 * ps + rp + x);
        }
#pragma unroll
        for (int pl = 0; pl < 12; ++pl) l[pl] = ld(lam1 + pl * ps + row + x);
        double h, qx, qy, e[12], mu[3];
        moments2d(v, h, qx, qy);
        feq2d<T>(h, qx, qy, P, e);
        adj_mu(l, h, qx, qy, P, mu[0], mu[1], mu[2]);
#pragma unroll
        for (int pl = 0; pl < 12; ++pl) acc += l[pl] * (e[pl] - v[pl]);
        const double oms = 1.0 - P.s;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            TA *b = lam0 + (4 * k) * ps;
            sth<2>(b + row + xm, oms * l[4 * k + 0] + P.s * mu[k]);
            sth<2>(b + ps + rm + x, oms * l[4 * k + 1] + P.s * mu[k]);
            sth<2>(b + 2 * ps + row + xp, oms * l[4 * k + 2] + P.s * mu[k]);
            sth<2>(b + 3 * ps + rp + x, oms * l[4 * k + 3] + P.s * mu[k]);
        }
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] += sh[0];
}

// ---- faces other than periodic ------------------------------------------------
// The transpose of a pull with face rules sends vt_p(x) to the slot the pull of
// population p at x read: the upstream node x - e_p inside the domain (or across
// a periodic face); across a Neumann face the node's own p; across a wall the
// node's own opposite population, negated for the momentum normal to the face;
// across an inflow face nowhere (the ghost is a constant).  Every slot then has
// one writer, except slot (p, y) of a node whose -e_p side is a Neumann face: it
// receives the push from y + e_p and y's own vt_p.  The own value goes to a small
// per-face buffer `side` (3 planes per face node in 2D, 2 in 1D) and a second
// kernel adds it in (a sum of two terms, so its order does not matter).  Slots
// (p, y) whose +e_p side is a Neumann or inflow face receive nothing: zero.
// side[(face * side_len + pos) * 3 + k], pos = the node's position along the face.

// Push of vt for plane pl = 4k + j (direction j: 0 +x, 1 +y, 2 -x, 3 -y) at (x, y).
template <typename TA>
__device__ __forceinline__ void adj_push2d(TA *__restrict__ lam0, double *__restrict__ side,
                                           int side_len, const Geo &G, int k, int j, int x, int y,
                                           double vt)
{
    const int pl = 4 * k + j;
    int sx = x - (j == 0 ? 1 : (j == 2 ? -1 : 0));
    int sy = y - (j == 1 ? 1 : (j == 3 ? -1 : 0));
    const int face = sx < 0 ? 0 : (sx >= G.nx ? 1 : (sy < 0 ? 2 : (sy >= G.ny ? 3 : -1)));
    if (face >= 0) {
        const int bc = G.bc[face];
        if (bc == BC_NEUMANN) {
            side[((long)face * side_len + (face < 2 ? y : x)) * 3 + k] = vt;
            return;
        }
        if (bc == BC_WALL) {
            const int opp = 4 * k + ((j + 2) & 3);
            const int normal = face < 2 ? 1 : 2;
            st(lam0 + opp * G.ps + (long)y * G.nx + x, k == normal ? -vt : vt);
            return;
        }
        if (bc != BC_PERIODIC) return;  // inflow
        sx = sx < 0 ? sx + G.nx : (sx >= G.nx ? sx - G.nx : sx);
        sy = sy < 0 ? sy + G.ny : (sy >= G.ny ? sy - G.ny : sy);
    }
    st(lam0 + pl * G.ps + (long)sy * G.nx + sx, vt);
}

template <typename T, typename TA>
__global__ void __launch_bounds__(256) k_adj2d_bnd(const T *__restrict__ un,
                                                   const TA *__restrict__ lam1, TA *__restrict__ lam0,
                                                   double *__restrict__ partials,
                                                   double *__restrict__ side, int side_len, Geo G,
                                                   Phys P, int tiles_x)
{
    __shared__ double sh[256];
    const int y = blockIdx.x / tiles_x;
    const int x = (blockIdx.x - y * tiles_x) * 256 + threadIdx.x;
    double acc = 0.0;
    if (x < G.nx) {
        const long row = (long)y * G.nx;
        double v[12], l[12];
        pull2d_generic(un, G, P, x, y, v);
#pragma unroll
        for (int pl = 0; pl < 12; ++pl) l[pl] = ld(lam1 + pl * G.ps + row + x);
        double h, qx, qy, e[12], mu[3];
        moments2d(v, h, qx, qy);
        feq2d<T>(h, qx, qy, P, e);
        adj_mu(l, h, qx, qy, P, mu[0], mu[1], mu[2]);
#pragma unroll
        for (int pl = 0; pl < 12; ++pl) acc += l[pl] * (e[pl] - v[pl]);
        const double oms = 1.0 - P.s;
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                adj_push2d(lam0, side, side_len, G, k, j, x, y, oms * l[4 * k + j] + P.s * mu[k]);
        // slots whose +e_j side is a Neumann or inflow face receive nothing
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int tx = x + (j == 0 ? 1 : (j == 2 ? -1 : 0));
            const int ty = y + (j == 1 ? 1 : (j == 3 ? -1 : 0));
            const int face =
                tx < 0 ? 0 : (tx >= G.nx ? 1 : (ty < 0 ? 2 : (ty >= G.ny ? 3 : -1)));
            if (face >= 0 && (G.bc[face] == BC_NEUMANN || G.bc[face] == BC_INFLOW)) {
#pragma unroll
                for (int k = 0; k < 3; ++k) st(lam0 + (4 * k + j) * G.ps + row + x, 0.0);
            }
        }
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] += sh[0];
}

// 1D: planes f+ (0), f- (1), g+ (2), g- (3); face 0 = x-, face 1 = x+.  With
// u = q / h and c = 1/(2 lambda), the partial derivatives of the a = 0 equilibria
// (Sec. 2 potentials) give
//   mu_h = (L_f+ + L_f-) / 2 + c (g h - u^2) (L_g+ - L_g-)
//   mu_q = c (L_f+ - L_f-) + (L_g+ + L_g-) / 2 + 2 u c (L_g+ - L_g-)
__device__ __forceinline__ void adj_mu1d(const double *l, double h, double q, const Phys &P,
                                         double &mh, double &mq)
{
    const double u = q * (1.0 / h);
    const double L1g = l[2] - l[3];
    mh = 0.5 * (l[0] + l[1]) + P.c * (P.g * h - u * u) * L1g;
    mq = P.c * (l[0] - l[1]) + 0.5 * (l[2] + l[3]) + 2.0 * u * P.c * L1g;
}

template <typename T, typename TA>
__global__ void __launch_bounds__(256) k_adj1d(const T *__restrict__ un,
                                               const TA *__restrict__ lam1, TA *__restrict__ lam0,
                                               double *__restrict__ partials,
                                               double *__restrict__ side, int side_len, Geo G,
                                               Phys P)
{
    __shared__ double sh[256];
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int nx = G.nx;
    const long ps = G.ps;
    double acc = 0.0;
    if (x < nx) {
        double v[4], l[4];
        pull1d(un, G, P, x, v);
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) l[pl] = ld(lam1 + pl * ps + x);
        double h, q, e[4], mu[2];
        moments1d(v, h, q);
        feq1d<T>(h, q, P, e);
        adj_mu1d(l, h, q, P, mu[0], mu[1]);
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) acc += l[pl] * (e[pl] - v[pl]);
        const double oms = 1.0 - P.s;
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) {
            const int k = pl >> 1;
            const double vt = oms * l[pl] + P.s * mu[k];
            const bool plus = (pl & 1) == 0;  // f+, g+ pull from x - 1
            int sx = plus ? x - 1 : x + 1;
            const int face = sx < 0 ? 0 : (sx >= nx ? 1 : -1);
            if (face >= 0) {
                const int bc = G.bc[face];
                if (bc == BC_NEUMANN) {
                    side[((long)face * side_len) * 3 + k] = vt;
                    continue;
                }
                if (bc == BC_WALL) {
                    st(lam0 + (pl ^ 1) * ps + x, k == 1 ? -vt : vt);
                    continue;
                }
                if (bc != BC_PERIODIC) continue;  // inflow
                sx = face == 0 ? nx - 1 : 0;
            }
            st(lam0 + pl * ps + sx, vt);
        }
        // slots whose +e side is a Neumann or inflow face receive nothing
        if (x == nx - 1 && (G.bc[1] == BC_NEUMANN || G.bc[1] == BC_INFLOW)) {
            st(lam0 + x, 0.0);
            st(lam0 + 2 * ps + x, 0.0);
        }
        if (x == 0 && (G.bc[0] == BC_NEUMANN || G.bc[0] == BC_INFLOW)) {
            st(lam0 + ps + x, 0.0);
            st(lam0 + 3 * ps + x, 0.0);
        }
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] += sh[0];
}

// Adds the Neumann faces' own contributions (side) into lam0: thread i of face
// `face` handles position i / ncomp, component i % ncomp.
template <typename TA>
__global__ void __launch_bounds__(256) k_adj_neumann(TA *__restrict__ lam0,
                                                     const double *__restrict__ side,
                                                     int side_len, Geo G, int dim, int face)
{
    const int ncomp = dim == 1 ? 2 : 3;
    const int len = dim == 1 ? 1 : (face < 2 ? G.ny : G.nx);
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= len * ncomp) return;
    const int pos = i / ncomp, k = i - pos * ncomp;
    long node;
    int pl;
    if (dim == 1) {
        node = face == 0 ? 0 : G.nx - 1;
        pl = 2 * k + face;  // f+ / g+ cross the x- face, f- / g- the x+ face
    } else {
        const int x = face == 0 ? 0 : (face == 1 ? G.nx - 1 : pos);
        const int y = face == 2 ? 0 : (face == 3 ? G.ny - 1 : pos);
        node = (long)y * G.nx + x;
        const int j = face == 0 ? 0 : (face == 1 ? 2 : (face == 2 ? 1 : 3));
        pl = 4 * k + j;
    }
    TA *p = lam0 + pl * G.ps + node;
    st(p, ld(p) + side[((long)face * side_len + pos) * 3 + k]);
}

// dL/du^T from dL/dh: the h planes (2D 0..3, 1D 0..1) take dL/dh, the rest 0.
template <typename T>
__global__ void __launch_bounds__(256) k_adj_terminal(const double *__restrict__ dLdh,
                                                      T *__restrict__ lam, Geo G, int dim)
{
    const long n = (long)G.nx * G.ny;
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double d = dLdh[i];
    const int nh = dim == 1 ? 2 : 4, np = dim == 1 ? 4 : 12;
    for (int pl = 0; pl < np; ++pl) st(lam + pl * G.ps + i, pl < nh ? d : 0.0);
}

template <typename T>
__global__ void __launch_bounds__(256) k_adj_grad_w0(const T *__restrict__ lam0,
                                                     const double *__restrict__ h0,
                                                     const double *__restrict__ qx0,
                                                     const double *__restrict__ qy0,
                                                     double *__restrict__ gh,
                                                     double *__restrict__ gqx,
                                                     double *__restrict__ gqy, Geo G, Phys P,
                                                     int dim)
{
    const long n = (long)G.nx * G.ny;
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    if (dim == 1) {
        double l[4], mh, mq;
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) l[pl] = ld(lam0 + pl * G.ps + i);
        adj_mu1d(l, h0[i], qx0 ? qx0[i] : 0.0, P, mh, mq);
        if (gh) gh[i] = mh;
        if (gqx) gqx[i] = mq;
        return;
    }
    double l[12];
#pragma unroll
    for (int pl = 0; pl < 12; ++pl) l[pl] = ld(lam0 + pl * G.ps + i);
    double mh, mx, my;
    adj_mu(l, h0[i], qx0 ? qx0[i] : 0.0, qy0 ? qy0[i] : 0.0, P, mh, mx, my);
    if (gh) gh[i] = mh;
    if (gqx) gqx[i] = mx;
    if (gqy) gqy[i] = my;
}

long adjoint_blocks(const Geo &G)
{
    const int tiles_x = (G.nx + 255) / 256;
    return (long)tiles_x * G.ny;
}

static bool geo_periodic(const Geo &G)
{
    return G.bc[0] == BC_PERIODIC && G.bc[1] == BC_PERIODIC && G.bc[2] == BC_PERIODIC &&
           G.bc[3] == BC_PERIODIC;
}

template <typename T, typename TA>
static void adj_launch(int dim, const void *un, const void *lam1, void *lam0, double *partials,
                       double *side, int side_len, const Geo &G, const Phys &P, hipStream_t st)
{
    const int tiles_x = (G.nx + 255) / 256;
    if (dim == 1)
        hipLaunchKernelGGL((k_adj1d<T, TA>), dim3(tiles_x), dim3(256), 0, st, (const T *)un,
                           (const TA *)lam1, (TA *)lam0, partials, side, side_len, G, P);
    else if (geo_periodic(G))
        hipLaunchKernelGGL((k_adj2d<T, TA>), dim3(tiles_x * G.ny), dim3(256), 0, st,
                           (const T *)un, (const TA *)lam1, (TA *)lam0, partials, G, P, tiles_x,
                           tiles_x * G.ny);
    else
        hipLaunchKernelGGL((k_adj2d_bnd<T, TA>), dim3(tiles_x * G.ny), dim3(256), 0, st,
                           (const T *)un, (const TA *)lam1, (TA *)lam0, partials, side, side_len,
                           G, P, tiles_x);
    // the Neumann faces' own contributions, after the pushes
    const int nf = dim == 1 ? 2 : 4;
    for (int face = 0; face < nf; ++face) {
        if (G.bc[face] != BC_NEUMANN) continue;
        const int len = (dim == 1 ? 1 : (face < 2 ? G.ny : G.nx)) * (dim == 1 ? 2 : 3);
        hipLaunchKernelGGL((k_adj_neumann<TA>), dim3((len + 255) / 256), dim3(256), 0, st,
                           (TA *)lam0, side, side_len, G, dim, face);
    }
}

int adjoint_side_len(const Geo &G) { return G.nx > G.ny ? G.nx : G.ny; }

hipError_t launch_adjoint(int dim, bool f32, bool a32, const void *un, const void *lam1,
                          void *lam0, double *partials, double *side, const Geo &G,
                          const Phys &P, hipStream_t st)
{
    const int side_len = adjoint_side_len(G);
    if (f32 && a32)
        adj_launch<float, float>(dim, un, lam1, lam0, partials, side, side_len, G, P, st);
    else if (f32)
        adj_launch<float, double>(dim, un, lam1, lam0, partials, side, side_len, G, P, st);
    else
        adj_launch<double, double>(dim, un, lam1, lam0, partials, side, side_len, G, P, st);
    return hipGetLastError();
}

hipError_t launch_adjoint_terminal(int dim, bool f32, const double *dLdh, void *lam,
                                   const Geo &G, hipStream_t st)
{
    const int nb = (int)(((long)G.nx * G.ny + 255) / 256);
    if (f32)
        hipLaunchKernelGGL(k_adj_terminal<float>, dim3(nb), dim3(256), 0, st, dLdh,
                           (float *)lam, G, dim);
    else
        hipLaunchKernelGGL(k_adj_terminal<double>, dim3(nb), dim3(256), 0, st, dLdh,
                           (double *)lam, G, dim);
    return hipGetLastError();
}

hipError_t launch_adjoint_grad_w0(int dim, bool f32, const void *lam0, const double *h0,
                                  const double *qx0, const double *qy0, double *gh, double *gqx,
                                  double *gqy, const Geo &G, const Phys &P, hipStream_t st)
{
    const int nb = (int)(((long)G.nx * G.ny + 255) / 256);
    if (f32)
        hipLaunchKernelGGL(k_adj_grad_w0<float>, dim3(nb), dim3(256), 0, st,
                           (const float *)lam0, h0, qx0, qy0, gh, gqx, gqy, G, P, dim);
    else
        hipLaunchKernelGGL(k_adj_grad_w0<double>, dim3(nb), dim3(256), 0, st,
                           (const double *)lam0, h0, qx0, qy0, gh, gqx, gqy, G, P, dim);
    return hipGetLastError();
}

} // namespace lbm
