// Discrete adjoint of the fused stream + collide step (2D, periodic faces).
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

template <typename T>
__global__ void __launch_bounds__(256) k_adj_terminal(const double *__restrict__ dLdh,
                                                      T *__restrict__ lam, Geo G)
{
    const long n = (long)G.nx * G.ny;
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double d = dLdh[i];
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) st(lam + pl * G.ps + i, d);
#pragma unroll
    for (int pl = 4; pl < 12; ++pl) st(lam + pl * G.ps + i, 0.0);
}

template <typename T>
__global__ void __launch_bounds__(256) k_adj_grad_w0(const T *__restrict__ lam0,
                                                     const double *__restrict__ h0,
                                                     const double *__restrict__ qx0,
                                                     const double *__restrict__ qy0,
                                                     double *__restrict__ gh,
                                                     double *__restrict__ gqx,
                                                     double *__restrict__ gqy, Geo G, Phys P)
{
    const long n = (long)G.nx * G.ny;
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
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

hipError_t launch_adjoint(bool f32, bool a32, const void *un, const void *lam1, void *lam0,
                          double *partials, const Geo &G, const Phys &P, hipStream_t st)
{
    const int tiles_x = (G.nx + 255) / 256;
    const int ntiles = tiles_x * G.ny;
    if (f32 && a32)
        hipLaunchKernelGGL((k_adj2d<float, float>), dim3(ntiles), dim3(256), 0, st,
                           (const float *)un, (const float *)lam1, (float *)lam0, partials, G, P,
                           tiles_x, ntiles);
    else if (f32)
        hipLaunchKernelGGL((k_adj2d<float, double>), dim3(ntiles), dim3(256), 0, st,
                           (const float *)un, (const double *)lam1, (double *)lam0, partials, G,
                           P, tiles_x, ntiles);
    else
        hipLaunchKernelGGL((k_adj2d<double, double>), dim3(ntiles), dim3(256), 0, st,
                           (const double *)un, (const double *)lam1, (double *)lam0, partials, G,
                           P, tiles_x, ntiles);
    return hipGetLastError();
}

hipError_t launch_adjoint_terminal(bool f32, const double *dLdh, void *lam, const Geo &G,
                                   hipStream_t st)
{
    const int nb = (int)(((long)G.nx * G.ny + 255) / 256);
    if (f32)
        hipLaunchKernelGGL(k_adj_terminal<float>, dim3(nb), dim3(256), 0, st, dLdh,
                           (float *)lam, G);
    else
        hipLaunchKernelGGL(k_adj_terminal<double>, dim3(nb), dim3(256), 0, st, dLdh,
                           (double *)lam, G);
    return hipGetLastError();
}

hipError_t launch_adjoint_grad_w0(bool f32, const void *lam0, const double *h0,
                                  const double *qx0, const double *qy0, double *gh, double *gqx,
                                  double *gqy, const Geo &G, const Phys &P, hipStream_t st)
{
    const int nb = (int)(((long)G.nx * G.ny + 255) / 256);
    if (f32)
        hipLaunchKernelGGL(k_adj_grad_w0<float>, dim3(nb), dim3(256), 0, st,
                           (const float *)lam0, h0, qx0, qy0, gh, gqx, gqy, G, P);
    else
        hipLaunchKernelGGL(k_adj_grad_w0<double>, dim3(nb), dim3(256), 0, st,
                           (const double *)lam0, h0, qx0, qy0, gh, gqx, gqy, G, P);
    return hipGetLastError();
}

} // namespace lbm
