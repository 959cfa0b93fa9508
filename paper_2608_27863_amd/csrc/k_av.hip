// Artificial viscosity (eq. av-coeffs and the smoothing operator S_h): the raw
// elemental viscosity from a bounded compression sensor with a Ducros-type
// vortical suppression, then averaging to a continuous field.
//
// At every Gauss-Lobatto node of an element, from the state u and its
// gradient q (q_{c,j} = du_c/dx_j):
//   dv_i/dx_j = (q_{1+i,j} - v_i q_{0,j}) / rho,  div = dv_k/dx_k,
//   omega = |curl v|,  c* = sqrt(gamma p* / rho*) with rho* = max(rho, rho_min),
//   p* = max(p, p_min) (the regularised thermodynamic state),
//   Ld = L(-div) (compression, limited to [0, inf)),  Lw = L(omega),
//   s = sqrt(h_m / k) Ld / c* * Ld^2 / (Ld^2 + Lw^2 + eps),
//   nu = c_av L(s),  L(s) limited to [0, s_max];
// the raw elemental value is the maximum over the element's nodes.
// Smoothing: vertex value = mean of the elemental values of the elements that
// share the vertex (periodic pairs identified), element value = mean of its 8
// vertex values, repeated; the field is the trilinear interpolant of the last
// vertex values at each element's nodes (continuous across faces).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "hdg_internal.h"

namespace hdg {
namespace {

struct GllNodes {
    double r[4][5];  // Gauss-Lobatto nodes of degree 1..4
};

__global__ void __launch_bounds__(256) k_av_raw(DevMesh dm, double gamma, AvParams ap, const double *__restrict__ U,
                                                const double *__restrict__ Q, double *__restrict__ nu_elem) {
    const int e = blockIdx.x;
    const int p = dm.elem_p[e], Np = (p + 1) * (p + 1) * (p + 1);
    const int64_t o = dm.node_off[e];
    const double *u = U + 5 * o, *q = Q + 15 * o;
    const double hk = sqrt(ap.h_m / (double)p);
    double best = 0.0;
    for (int i = threadIdx.x; i < Np; i += blockDim.x) {
        const double rho = u[i];
        double v[3];
        for (int a = 0; a < 3; ++a) v[a] = u[(1 + a) * Np + i] / rho;
        const double pr = (gamma - 1.0) * (u[4 * Np + i] - 0.5 * rho * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]));
        double dv[3][3];
        for (int a = 0; a < 3; ++a)
            for (int j = 0; j < 3; ++j) dv[a][j] = (q[(3 * (1 + a) + j) * Np + i] - v[a] * q[j * Np + i]) / rho;
        const double div = dv[0][0] + dv[1][1] + dv[2][2];
        const double w0 = dv[2][1] - dv[1][2], w1 = dv[0][2] - dv[2][0], w2 = dv[1][0] - dv[0][1];
        const double om = sqrt(w0 * w0 + w1 * w1 + w2 * w2);
        const double cs = sqrt(gamma * fmax(pr, ap.p_min) / fmax(rho, ap.rho_min));
        const double Ld = fmax(-div, 0.0), Lw = fmax(om, 0.0);
        const double s = hk * Ld / cs * (Ld * Ld) / (Ld * Ld + Lw * Lw + ap.eps);
        const double val = ap.c_av * fmin(fmax(s, 0.0), ap.s_max);
        best = fmax(best, val);
    }
    __shared__ double red[256];
    red[threadIdx.x] = best;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) nu_elem[e] = red[0];
}

// vertex class k: mean over the elements touching it (ascending element order)
__global__ void __launch_bounds__(256) k_av_vertex(DevMesh dm, const double *__restrict__ nu_elem,
                                                   double *__restrict__ nu_vert) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= dm.n_vclass) return;
    const int s0 = dm.av_src_ptr[k], s1 = dm.av_src_ptr[k + 1];
    double acc = 0.0;
    for (int s = s0; s < s1; ++s) acc += nu_elem[dm.av_src[s]];
    nu_vert[k] = acc / (double)(s1 - s0);
}

__global__ void __launch_bounds__(256) k_av_elem(DevMesh dm, const double *__restrict__ nu_vert,
                                                 double *__restrict__ nu_elem) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= dm.n_elem) return;
    double acc = 0.0;
    for (int c = 0; c < 8; ++c) acc += nu_vert[dm.av_corner[8 * e + c]];
    nu_elem[e] = acc / 8.0;
}

// nodal field: trilinear interpolant of the element's 8 corner values
__global__ void __launch_bounds__(128) k_av_nodes(DevMesh dm, GllNodes gn, const double *__restrict__ nu_vert,
                                                  double *__restrict__ nu) {
    const int e = blockIdx.x;
    const int p = dm.elem_p[e], n1 = p + 1, Np = n1 * n1 * n1;
    double cv[8];
    for (int c = 0; c < 8; ++c) cv[c] = nu_vert[dm.av_corner[8 * e + c]];
    for (int i = threadIdx.x; i < Np; i += blockDim.x) {
        const double x[3] = {gn.r[p - 1][i % n1], gn.r[p - 1][(i / n1) % n1], gn.r[p - 1][i / (n1 * n1)]};
        double acc = 0.0;
        for (int c = 0; c < 8; ++c) {
            double w = 1.0;
            for (int d = 0; d < 3; ++d) w *= ((c >> d) & 1) ? 0.5 * (1.0 + x[d]) : 0.5 * (1.0 - x[d]);
            acc += w * cv[c];
        }
        nu[dm.node_off[e] + i] = acc;
    }
}

// constant element value at the nodes (no smoothing)
__global__ void __launch_bounds__(128) k_av_const(DevMesh dm, const double *__restrict__ nu_elem,
                                                  double *__restrict__ nu) {
    const int e = blockIdx.x;
    const int p = dm.elem_p[e], Np = (p + 1) * (p + 1) * (p + 1);
    for (int i = threadIdx.x; i < Np; i += blockDim.x) nu[dm.node_off[e] + i] = nu_elem[e];
}

__global__ void __launch_bounds__(256) k_copy_n(const double *__restrict__ a, double *__restrict__ b, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

}  // namespace

size_t av_work_bytes(const hdg_ctx *ctx) {
    return sizeof(double) * ((size_t)(ctx->n_elem + 31) / 32 * 32 + (size_t)ctx->n_vclass) + 256;
}

int launch_av_field(const hdg_ctx *ctx, const AvParams &ap, const double *U, const double *Q, double *nu_raw,
                    double *nu, void *work, hipStream_t s) {
    const DevMesh &dm = ctx->dm;
    double *el = (double *)work;
    double *vt = el + (size_t)(ctx->n_elem + 31) / 32 * 32;
    GllNodes gn{};
    for (int p = 1; p <= kMaxP; ++p) gll_nodes(p, gn.r[p - 1]);
    const int ne = ctx->n_elem, nv = ctx->n_vclass;
    hipLaunchKernelGGL(k_av_raw, dim3(ne), dim3(256), 0, s, dm, ctx->phys.gamma, ap, U, Q, el);
    if (nu_raw) hipLaunchKernelGGL(k_copy_n, dim3((ne + 255) / 256), dim3(256), 0, s, (const double *)el, nu_raw, ne);
    if (ap.smooth_iters == 0) {
        hipLaunchKernelGGL(k_av_const, dim3(ne), dim3(128), 0, s, dm, (const double *)el, nu);
        return (int)hipGetLastError();
    }
    for (int it = 0; it < ap.smooth_iters; ++it) {
        hipLaunchKernelGGL(k_av_vertex, dim3((nv + 255) / 256), dim3(256), 0, s, dm, (const double *)el, vt);
        if (it + 1 < ap.smooth_iters)
            hipLaunchKernelGGL(k_av_elem, dim3((ne + 255) / 256), dim3(256), 0, s, dm, (const double *)vt, el);
    }
    hipLaunchKernelGGL(k_av_nodes, dim3(ne), dim3(128), 0, s, dm, gn, (const double *)vt, nu);
    return (int)hipGetLastError();
}

}  // namespace hdg
