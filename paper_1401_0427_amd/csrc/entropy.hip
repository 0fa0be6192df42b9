// Discrete microscopic entropy H(f) = sum over nodes and populations of h_j(f_j)
// (Sec. 1), the Legendre dual of the Perthame-Bouchut potentials of the a = 0
// lattices (Sec. 2, eq. 2-potentiels-st-venant-1d-suite; Sec. 3, eqs.
// 3-st-venant-contraintes-2 and 3-st-venant-enplus):
//   h_j^*(theta, U) = w K P^2 (1 + sigma kappa xi),  P = theta + |U|^2 / 2,
// with K = 1/(2g), xi the velocity component along e_j = sigma * axis,
// (w, kappa) = (1/2, 1/lambda) in 1D and (1/4, 2/lambda) in 2D.
//
// For one population with density component f > 0, momentum component g_xi
// along its axis and g_om across it, the stationarity conditions
// grad h_j^*(phi) = (f, g_xi, g_om) reduce in closed form to
//   om = g_om / f,   P = f / (2 w K D),   D = 1 + kappa z,   z = sigma xi,
//   S(z) = z f + A / D^2 - sigma g_xi = 0,   A = kappa f^2 / (4 w K),
// and then
//   h_j = A (1 + 2 kappa z) / (kappa D^2) + (z^2 + om^2) f / 2.
// The Hessian of h_j^* is positive definite at such a point exactly when
// D > Dc = (2 kappa A / f)^(1/3), i.e. S'(z) > 0 (its Schur complement with
// respect to theta is diag(P D - P^2 kappa^2 / D, P D)).  S is convex and, for
// D > Dc, increasing, so it has at most one root there; Newton's method
// started to the right of it (S > 0) decreases monotonically onto it, and an
// iterate that falls to D <= Dc shows that there is none: the population is
// then outside the domain of the dual, counted as invalid, and its node's
// entropy is +infinity.
#include "internal.h"

namespace lbm {

struct EntPop {
    double h;
    int ok;
};

// cA = kappa / (4 w K) and ik = 1 / kappa are per-lattice constants (A = cA f^2).
// Each Newton iteration takes one reciprocal of D and one quotient; the step
// tests compare |dz| with (1 + |z|) by multiplication instead of dividing.
__device__ __forceinline__ EntPop ent_pop(double f, double gxi, double gom, double sigma,
                                          double cA, double kappa, double ik)
{
    EntPop r = {0.0, 0};
    if (!(f > 0.0)) return r;
    const double rf = 1.0 / f;
    const double om = gom * rf;
    const double A = cA * (f * f);
    const double tkA = 2.0 * kappa * A;
    const double gs = sigma * gxi;
    const double Dc = cbrt(tkA * rf);
    const double zc = (Dc - 1.0) * ik;
    // start right of the root: from max(zc, first-order guess), then outwards
    double z = fmax(zc, (gs - A) * rf);
    double step = fmax(fabs(z), ik);
    double S = 0.0;
    for (int k = 0; k < 200; ++k) {
        const double iD = 1.0 / (1.0 + kappa * z);
        S = z * f + A * (iD * iD) - gs;
        if (S > 0.0) break;
        z += step;
        step *= 2.0;
    }
    if (!(S > 0.0)) return r;
    // relative step |dz| / (1 + |z|) of the previous iteration, as the pair (a, b)
    double pa = 1.0, pb = 0.0;
    int conv = 0;
    for (int it = 0; it < 100; ++it) {
        const double iD = 1.0 / (1.0 + kappa * z);
        const double iD2 = iD * iD;
        const double Sz = z * f + A * iD2 - gs;
        const double dS = f - tkA * (iD2 * iD);
        if (!(dS > 0.0)) break;
        const double dz = Sz / dS;
        z -= dz;
        if (!(z > zc)) break;  // no root with D > Dc
        const double a = fabs(dz), b = 1.0 + fabs(z);
        // converged: relative step <= 1e-15, or below 1e-10 and no longer shrinking
        if (a <= 1e-15 * b || (a < 1e-10 * b && a * pb >= pa * b)) {
            conv = 1;
            break;
        }
        pa = a;
        pb = b;
    }
    if (!conv) return r;
    const double iD = 1.0 / (1.0 + kappa * z);
    const double iD2 = iD * iD;
    if (!(f - tkA * (iD2 * iD) > 0.0)) return r;
    r.h = A * (1.0 + 2.0 * kappa * z) * iD2 * ik + 0.5 * (z * z + om * om) * f;
    r.ok = 1;
    return r;
}

// Fixed-order tree sum of two values over a 256-thread workgroup.
__device__ __forceinline__ void ent_block_sum(double (*sh)[256], double *v)
{
    const int t = threadIdx.x;
    sh[0][t] = v[0];
    sh[1][t] = v[1];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) {
            sh[0][t] = sh[0][t] + sh[0][t + s];
            sh[1][t] = sh[1][t] + sh[1][t + s];
        }
        __syncthreads();
    }
    v[0] = sh[0][0];
    v[1] = sh[1][0];
}

template <typename T>
__global__ void __launch_bounds__(256) k_entropy(int dim, const T *__restrict__ state, Geo G,
                                                 double lambda, double g,
                                                 double *__restrict__ h_node,
                                                 double *__restrict__ partials)
{
    __shared__ double sh[2][256];
    const long n = (long)G.nx * G.ny;
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    const double K = 0.5 / g;
    double v[2] = {0.0, 0.0};  // node entropy, invalid populations
    if (i < n) {
        double H = 0.0;
        int bad = 0;
        if (dim == 1) {
            // planes f+, f-, g+, g-
            const double kappa = 1.0 / lambda;
            const double cA = kappa / (4.0 * 0.5 * K);
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const double f = ld(state + j * G.ps + i);
                const double q = ld(state + (2 + j) * G.ps + i);
                const EntPop e = ent_pop(f, q, 0.0, j == 0 ? 1.0 : -1.0, cA, kappa, lambda);
                H += e.h;
                bad += 1 - e.ok;
            }
        } else {
            // planes (h: e1..e4, qx: e1..e4, qy: e1..e4); e1 = +x, e2 = +y, e3 = -x, e4 = -y
            const double kappa = 2.0 / lambda;
            const double cA = kappa / (4.0 * 0.25 * K);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double f = ld(state + j * G.ps + i);
                const double gx = ld(state + (4 + j) * G.ps + i);
                const double gy = ld(state + (8 + j) * G.ps + i);
                const bool xaxis = (j & 1) == 0;
                const EntPop e = ent_pop(f, xaxis ? gx : gy, xaxis ? gy : gx, j < 2 ? 1.0 : -1.0,
                                         cA, kappa, 0.5 * lambda);
                H += e.h;
                bad += 1 - e.ok;
            }
        }
        if (bad) H = INFINITY;
        if (h_node) h_node[i] = H;
        v[0] = H;
        v[1] = (double)bad;
    }
    if (partials) {
        ent_block_sum(sh, v);
        if (threadIdx.x == 0) {
            partials[(long)blockIdx.x * 2 + 0] = v[0];
            partials[(long)blockIdx.x * 2 + 1] = v[1];
        }
    }
}

hipError_t launch_entropy(int dim, bool f32, const void *state, const Geo &G, double lambda,
                          double g, double *h_node, double *partials, hipStream_t st,
                          int *nblocks_out)
{
    const long n = (long)G.nx * G.ny;
    const int nb = (int)((n + 255) / 256);
    if (nblocks_out) *nblocks_out = nb;
    if (f32)
        hipLaunchKernelGGL(k_entropy<float>, dim3(nb), dim3(256), 0, st, dim,
                           (const float *)state, G, lambda, g, h_node, partials);
    else
        hipLaunchKernelGGL(k_entropy<double>, dim3(nb), dim3(256), 0, st, dim,
                           (const double *)state, G, lambda, g, h_node, partials);
    return hipGetLastError();
}

} // namespace lbm
