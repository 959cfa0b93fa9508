// Host side of libhdg: context creation (quadrature tables, geometry,
// assembly maps, block-sparse pattern), layout queries, argument checks and
// the C-ABI entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <new>
#include <vector>

#include "hdg_internal.h"

using hdg::DevMesh;

namespace {

// ---------------------------------------------------------------- 1-D rules
// Legendre P_n and P_n' by the three-term recurrence.
void legendre(int n, double x, double &P, double &dP) {
    double pm1 = 1.0, p = x;
    if (n == 0) { P = 1.0; dP = 0.0; return; }
    for (int k = 1; k < n; ++k) {
        double pn = ((2 * k + 1) * x * p - k * pm1) / (k + 1);
        pm1 = p;
        p = pn;
    }
    P = p;
    dP = n * (x * p - pm1) / (x * x - 1.0);
}

void gauss_rule(int nq, double *x, double *w) {
    for (int i = 0; i < nq; ++i) {
        // initial guess from the asymptotic node location, ascending order
        double t = std::cos(M_PI * (nq - i - 0.25) / (nq + 0.5));
        for (int it = 0; it < 200; ++it) {
            double P, dP;
            legendre(nq, t, P, dP);
            double step = P / dP;
            t -= step;
            if (std::fabs(step) <= 1e-17) break;
        }
        double P, dP;
        legendre(nq, t, P, dP);
        x[i] = t;
        w[i] = 2.0 / ((1.0 - t * t) * dP * dP);
    }
}

// Gauss-Lobatto nodes: endpoints and the zeros of P_p', which are the Gauss
// points of the Jacobi weight (1-x^2); Newton on P_p' using
// P_p'' = (2x P_p' - p(p+1) P_p) / (1 - x^2).
void lobatto_nodes(int p, double *r) {
    r[0] = -1.0;
    r[p] = 1.0;
    for (int i = 1; i < p; ++i) {
        double t = -std::cos(M_PI * i / p);
        for (int it = 0; it < 200; ++it) {
            double P, dP;
            legendre(p, t, P, dP);
            double d2P = (2.0 * t * dP - p * (p + 1.0) * P) / (1.0 - t * t);
            double step = dP / d2P;
            t -= step;
            if (std::fabs(step) <= 1e-17) break;
        }
        r[i] = t;
    }
}

// Lagrange basis on nodes r[0..p] (barycentric form) and its derivative at t.
void lagrange_eval(int p, const double *r, double t, double *val, double *der) {
    double bw[8];
    for (int a = 0; a <= p; ++a) {
        double prod = 1.0;
        for (int b = 0; b <= p; ++b)
            if (b != a) prod *= (r[a] - r[b]);
        bw[a] = 1.0 / prod;
    }
    for (int a = 0; a <= p; ++a) {
        if (t == r[a]) {
            for (int b = 0; b <= p; ++b) val[b] = (b == a) ? 1.0 : 0.0;
            // derivative at a node: l_b'(r_a) = (bw_b / bw_a) / (r_a - r_b), l_a' = -sum_{b!=a}
            if (der) {
                double s = 0.0;
                for (int b = 0; b <= p; ++b) {
                    if (b == a) continue;
                    der[b] = (bw[b] / bw[a]) / (r[a] - r[b]);
                    s += der[b];
                }
                der[a] = -s;
            }
            return;
        }
    }
    double ell = 1.0;
    for (int b = 0; b <= p; ++b) ell *= (t - r[b]);
    double S1 = 0.0;
    for (int b = 0; b <= p; ++b) S1 += 1.0 / (t - r[b]);
    for (int a = 0; a <= p; ++a) {
        double v = ell * bw[a] / (t - r[a]);
        val[a] = v;
        // d/dt [ell(t) bw_a / (t - r_a)] = v * (S1 - 1/(t-r_a))
        if (der) der[a] = v * (S1 - 1.0 / (t - r[a]));
    }
}

void build_tables(double *T) {
    std::memset(T, 0, sizeof(double) * hdg::kTblSize);
    for (int nq = 3; nq <= 6; ++nq) {
        double x[8], w[8];
        gauss_rule(nq, x, w);
        for (int g = 0; g < nq; ++g) T[hdg::tbl_W(nq, g)] = w[g];
    }
    for (int p = 1; p <= hdg::kMaxP; ++p) {
        double r[8];
        lobatto_nodes(p, r);
        for (int q = 1; q <= hdg::kMaxP; ++q) {
            double x[8], w[8];
            gauss_rule(q + 2, x, w);
            for (int s = 0; s < q + 2; ++s) {
                double val[8], der[8];
                lagrange_eval(p, r, x[s], val, der);
                for (int a = 0; a <= p; ++a) {
                    T[hdg::tbl_L(p, q, a, s)] = val[a];
                    if (q == p) T[hdg::tbl_D(p, a, s)] = der[a];
                }
            }
        }
    }
}

// ---------------------------------------------------------------- geometry
// Trilinear map of the 8 vertices (tensor order): Jacobian J[i][d] = dx_i/dxi_d.
void map_jacobian(const double *X8, const double xi[3], double J[3][3]) {
    for (int i = 0; i < 3; ++i)
        for (int d = 0; d < 3; ++d) J[i][d] = 0.0;
    for (int v = 0; v < 8; ++v) {
        double f[3], df[3];
        for (int d = 0; d < 3; ++d) {
            double s = ((v >> d) & 1) ? 0.5 : -0.5;
            f[d] = 0.5 + s * xi[d];
            df[d] = s;
        }
        double g[3] = {df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]};
        for (int i = 0; i < 3; ++i)
            for (int d = 0; d < 3; ++d) J[i][d] += g[d] * X8[3 * v + i];
    }
}

// Triquadratic map of 27 nodes (tensor order, x fastest; reference
// coordinates -1, 0, 1 per direction): J[i][d] = dx_i/dxi_d.  The quadratic
// Lagrange factors on {-1, 0, 1}: l0 = t(t-1)/2, l1 = 1 - t^2, l2 = t(t+1)/2.
void map_jacobian27(const double *X27, const double xi[3], double J[3][3]) {
    double l[3][3], dl[3][3];
    for (int d = 0; d < 3; ++d) {
        const double t = xi[d];
        l[d][0] = 0.5 * t * (t - 1.0);
        l[d][1] = 1.0 - t * t;
        l[d][2] = 0.5 * t * (t + 1.0);
        dl[d][0] = t - 0.5;
        dl[d][1] = -2.0 * t;
        dl[d][2] = t + 0.5;
    }
    for (int i = 0; i < 3; ++i)
        for (int d = 0; d < 3; ++d) J[i][d] = 0.0;
    for (int c = 0; c < 3; ++c)
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a) {
                const double *X = X27 + 3 * (a + 3 * (b + 3 * c));
                const double g[3] = {dl[0][a] * l[1][b] * l[2][c], l[0][a] * dl[1][b] * l[2][c],
                                     l[0][a] * l[1][b] * dl[2][c]};
                for (int i = 0; i < 3; ++i)
                    for (int d = 0; d < 3; ++d) J[i][d] += g[d] * X[i];
            }
}

// Cofactor inverse: G = J^{-1}, returns det J.
double invert3(const double J[3][3], double G[3][3]) {
    double C[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            C[i][j] = J[i1][j1] * J[i2][j2] - J[i1][j2] * J[i2][j1];
        }
    double det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
    for (int d = 0; d < 3; ++d)
        for (int j = 0; j < 3; ++j) G[d][j] = C[j][d] / det;
    return det;
}

template <class T>
int upload(hdg_ctx *ctx, const std::vector<T> &h, const T **dst) {
    size_t bytes = std::max<size_t>(h.size(), 1) * sizeof(T);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return HDG_ERR_OUT_OF_MEMORY;
    ctx->allocations.push_back(p);
    if (!h.empty() && hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return HDG_ERR_DEVICE;
    *dst = static_cast<const T *>(p);
    return HDG_OK;
}

int trace_size(int pf) { return 5 * (pf + 1) * (pf + 1); }

}  // namespace

namespace hdg {
void gll_nodes(int p, double *r) { lobatto_nodes(p, r); }
}  // namespace hdg

// ====================================================================== API
extern "C" {

const char *hdg_status_string(int s) {
    switch (s) {
        case HDG_OK: return "ok";
        case HDG_ERR_INVALID_ARGUMENT: return "invalid argument";
        case HDG_ERR_UNSUPPORTED: return "unsupported";
        case HDG_ERR_OUT_OF_MEMORY: return "out of device memory";
        case HDG_ERR_DEVICE: return "HIP device error";
        case HDG_ERR_WORKSPACE: return "workspace too small";
        default: return "unknown status";
    }
}

void hdg_destroy(hdg_ctx *ctx) {
    if (!ctx) return;
    for (void *p : ctx->allocations) (void)hipFree(p);
    delete ctx;
}

int hdg_create(const hdg_mesh_desc *m, const hdg_phys *phys, hdg_ctx **out) {
    if (!m || !phys || !out) return HDG_ERR_INVALID_ARGUMENT;
    *out = nullptr;
    if (m->n_elem <= 0 || m->n_face <= 0 || m->n_vert <= 0 || !m->vert_xyz || !m->elem_vert ||
        !m->elem_face || !m->face_elem || !m->face_bc || !m->elem_p)
        return HDG_ERR_INVALID_ARGUMENT;
    if (!(phys->gamma > 1.0) || !(phys->prandtl > 0.0) || !(phys->reynolds > 0.0) || !(phys->mach > 0.0) ||
        !(phys->dt > 0.0) || !(phys->tau >= 0.0) || !(phys->alpha >= 0.0) ||
        (phys->visc_law != 0 && phys->visc_law != 1))
        return HDG_ERR_INVALID_ARGUMENT;
    const int ne = m->n_elem, nf = m->n_face;
    hdg_ctx *ctx = new (std::nothrow) hdg_ctx();
    if (!ctx) return HDG_ERR_OUT_OF_MEMORY;
    auto fail = [&](int st) { hdg_destroy(ctx); return st; };
    ctx->n_elem = ne;
    ctx->n_face = nf;
    ctx->phys = {phys->gamma, phys->prandtl, phys->reynolds, phys->mach, phys->tau, phys->dt, phys->alpha,
                 phys->visc_law};
    // ---- validate topology
    ctx->elem_p.resize(ne);
    for (int e = 0; e < ne; ++e) {
        int p = m->elem_p[e];
        if (p < 1 || p > hdg::kMaxP) return fail(HDG_ERR_INVALID_ARGUMENT);
        ctx->elem_p[e] = p;
        for (int v = 0; v < 8; ++v)
            if (m->elem_vert[8 * e + v] < 0 || m->elem_vert[8 * e + v] >= m->n_vert) return fail(HDG_ERR_INVALID_ARGUMENT);
    }
    ctx->elem_face.assign(m->elem_face, m->elem_face + 6 * ne);
    ctx->face_elem.assign(m->face_elem, m->face_elem + 4 * nf);
    ctx->face_bc.resize(nf);
    ctx->face_p.assign(nf, 0);
    for (int F = 0; F < nf; ++F) {
        ctx->face_bc[F] = m->face_bc[F];
        if (m->face_bc[F] < 0 || m->face_bc[F] > 5) return fail(HDG_ERR_INVALID_ARGUMENT);
        int e0 = ctx->face_elem[4 * F], l0 = ctx->face_elem[4 * F + 1];
        int e1 = ctx->face_elem[4 * F + 2], l1 = ctx->face_elem[4 * F + 3];
        if (e0 < 0 || e0 >= ne || l0 < 0 || l0 > 5) return fail(HDG_ERR_INVALID_ARGUMENT);
        if (ctx->elem_face[6 * e0 + l0] != F) return fail(HDG_ERR_INVALID_ARGUMENT);
        ctx->face_p[F] = ctx->elem_p[e0];
        if (e1 >= 0) {
            if (e1 >= ne || l1 < 0 || l1 > 5 || ctx->elem_face[6 * e1 + l1] != F) return fail(HDG_ERR_INVALID_ARGUMENT);
            if (l0 / 2 != l1 / 2 || l0 == l1) return fail(HDG_ERR_INVALID_ARGUMENT);  // opposite sides
            if (ctx->face_bc[F]) return fail(HDG_ERR_INVALID_ARGUMENT);
            ctx->face_p[F] = std::max(ctx->face_p[F], ctx->elem_p[e1]);
        } else if (!ctx->face_bc[F]) {
            return fail(HDG_ERR_INVALID_ARGUMENT);  // one-sided face must be a boundary face
        }
    }
    for (int e = 0; e < ne; ++e)
        for (int lf = 0; lf < 6; ++lf) {
            int F = ctx->elem_face[6 * e + lf];
            if (F < 0 || F >= nf) return fail(HDG_ERR_INVALID_ARGUMENT);
            bool ok = (ctx->face_elem[4 * F] == e && ctx->face_elem[4 * F + 1] == lf) ||
                      (ctx->face_elem[4 * F + 2] == e && ctx->face_elem[4 * F + 3] == lf);
            if (!ok) return fail(HDG_ERR_INVALID_ARGUMENT);
        }
    // ---- sizes and offsets
    ctx->node_off.assign(ne + 1, 0);
    ctx->E_off.assign(ne + 1, 0);
    ctx->SK_off.assign(ne + 1, 0);
    ctx->asm_off.assign(ne + 1, 0);
    ctx->qp_off.assign(ne + 1, 0);
    ctx->asmsys_off.assign(ne + 1, 0);
    ctx->tloc_off.assign(ne + 1, 0);
    ctx->m32_off.assign(ne + 1, 0);
    ctx->x_off.assign(ne + 1, 0);
    ctx->vgeo_off.assign(ne + 1, 0);
    ctx->fgeo_off.assign(6 * ne + 1, 0);
    ctx->toff.assign(7 * ne, 0);
    ctx->elem_n.resize(ne);
    ctx->elem_f.resize(ne);
    ctx->face_off.assign(nf + 1, 0);
    for (int F = 0; F < nf; ++F) {
        ctx->face_off[F + 1] = ctx->face_off[F] + trace_size(ctx->face_p[F]);
        if (trace_size(ctx->face_p[F]) % 16 != 0) ctx->face_cols_aligned = false;
    }
    for (int e = 0; e < ne; ++e) {
        int p = ctx->elem_p[e], Np = (p + 1) * (p + 1) * (p + 1), Nq = (p + 2) * (p + 2) * (p + 2);
        int n = 20 * Np, f = 0, nqf_tot = 0;
        for (int lf = 0; lf < 6; ++lf) {
            int pf = ctx->face_p[ctx->elem_face[6 * e + lf]];
            ctx->toff[7 * e + lf] = f;
            f += trace_size(pf);
            int nqf = (pf + 2) * (pf + 2);
            nqf_tot += nqf;
            ctx->fgeo_off[6 * e + lf + 1] = ctx->fgeo_off[6 * e + lf] + 4 * nqf;
        }
        ctx->toff[7 * e + 6] = f;
        ctx->elem_n[e] = n;
        ctx->elem_f[e] = f;
        if (f % 16 != 0) ctx->asm_cols_aligned64 = false;
        if (f % 32 != 0) ctx->asm_cols_aligned32 = false;
        if (p != ctx->elem_p[0]) ctx->uniform_p = false;
        ctx->max_n = std::max(ctx->max_n, n);
        ctx->max_f = std::max(ctx->max_f, f);
        ctx->max_p = std::max(ctx->max_p, p);
        ctx->node_off[e + 1] = ctx->node_off[e] + Np;
        ctx->E_off[e + 1] = ctx->E_off[e] + (int64_t)(n + f) * hdg::e_ld(n, f);
        ctx->SK_off[e + 1] = ctx->SK_off[e] + (int64_t)f * (f + 1);
        ctx->asm_off[e + 1] = (ctx->asm_off[e] + (int64_t)f * f + 31) / 32 * 32;  // blocks start on 128-byte lines
        ctx->qp_off[e + 1] = ctx->qp_off[e] + (int64_t)(hdg::kVJac + hdg::kVRes) * Nq + (int64_t)hdg::kFPer * nqf_tot;
        ctx->vgeo_off[e + 1] = ctx->vgeo_off[e] + 10 * Nq;
        const int fe = hdg::asm_pad(f);  // Schwarz system size
        ctx->asmsys_off[e + 1] = ctx->asmsys_off[e] + (int64_t)fe * hdg::e_ld(fe, fe);
        ctx->tloc_off[e + 1] = ctx->tloc_off[e] + f;
        ctx->m32_off[e + 1] = ctx->m32_off[e] + (int64_t)n * hdg::e_ld(n, f);
        ctx->x_off[e + 1] = ctx->x_off[e] + (int64_t)n * hdg::x_ld(f);
    }
    for (int F = 0; F < nf; ++F) ctx->max_b = std::max(ctx->max_b, trace_size(ctx->face_p[F]));
    // ---- tables and geometry
    std::vector<double> tbl(hdg::kTblSize);
    build_tables(tbl.data());
    std::vector<double> vgeo(ctx->vgeo_off[ne]), fgeo(ctx->fgeo_off[6 * ne]);
    for (int e = 0; e < ne; ++e) {
        double X8[24];
        for (int v = 0; v < 8; ++v)
            for (int i = 0; i < 3; ++i) X8[3 * v + i] = m->vert_xyz[3 * m->elem_vert[8 * e + v] + i];
        const double *X27 = m->elem_geom ? m->elem_geom + 81 * (size_t)e : nullptr;
        auto jac = [&](const double xi[3], double J[3][3]) {
            if (X27) map_jacobian27(X27, xi, J);
            else map_jacobian(X8, xi, J);
        };
        int p = ctx->elem_p[e], nq = p + 2, Nq = nq * nq * nq;
        double x[8], w[8];
        gauss_rule(nq, x, w);
        double *vg = vgeo.data() + ctx->vgeo_off[e];
        for (int g2 = 0; g2 < nq; ++g2)
            for (int g1 = 0; g1 < nq; ++g1)
                for (int g0 = 0; g0 < nq; ++g0) {
                    int g = g0 + nq * (g1 + nq * g2);
                    double xi[3] = {x[g0], x[g1], x[g2]}, J[3][3], G[3][3];
                    jac(xi, J);
                    double det = invert3(J, G);
                    if (!(det > 0.0)) return fail(HDG_ERR_INVALID_ARGUMENT);
                    vg[g] = w[g0] * w[g1] * w[g2] * det;
                    for (int d = 0; d < 3; ++d)
                        for (int j = 0; j < 3; ++j) vg[(1 + 3 * d + j) * Nq + g] = G[d][j];
                }
        for (int lf = 0; lf < 6; ++lf) {
            int d = lf / 2, t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
            double sgn = (lf & 1) ? 1.0 : -1.0;
            int pf = ctx->face_p[ctx->elem_face[6 * e + lf]], nqf1 = pf + 2, nqf = nqf1 * nqf1;
            double xf[8], wf[8];
            gauss_rule(nqf1, xf, wf);
            double *fg = fgeo.data() + ctx->fgeo_off[6 * e + lf];
            for (int s1 = 0; s1 < nqf1; ++s1)
                for (int s0 = 0; s0 < nqf1; ++s0) {
                    int s = s0 + nqf1 * s1;
                    double xi[3], J[3][3], G[3][3];
                    xi[d] = sgn;
                    xi[t0] = xf[s0];
                    xi[t1] = xf[s1];
                    jac(xi, J);
                    double det = invert3(J, G);
                    if (!(det > 0.0)) return fail(HDG_ERR_INVALID_ARGUMENT);
                    // Nanson: n dS = det J J^{-T} n_ref dS_ref, n_ref = sgn e_d
                    double N[3] = {sgn * det * G[d][0], sgn * det * G[d][1], sgn * det * G[d][2]};
                    double ws = wf[s0] * wf[s1];
                    for (int j = 0; j < 3; ++j) fg[j * nqf + s] = ws * N[j];
                    fg[3 * nqf + s] = ws * std::sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
                }
        }
    }
    // an element meeting the same face twice (one element across a periodic
    // direction) makes its Schwarz patch repeat unknowns
    for (int e = 0; e < ne; ++e)
        for (int a = 0; a < 6; ++a)
            for (int b = a + 1; b < 6; ++b)
                if (ctx->elem_face[6 * e + a] == ctx->elem_face[6 * e + b]) ctx->repeated_face = true;
    // ---- block-sparse pattern and gather lists
    std::vector<std::vector<int>> cols(nf);
    for (int e = 0; e < ne; ++e)
        for (int a = 0; a < 6; ++a)
            for (int b = 0; b < 6; ++b) cols[ctx->elem_face[6 * e + a]].push_back(ctx->elem_face[6 * e + b]);
    ctx->bsr_row_ptr.assign(nf + 1, 0);
    for (int F = 0; F < nf; ++F) {
        std::sort(cols[F].begin(), cols[F].end());
        cols[F].erase(std::unique(cols[F].begin(), cols[F].end()), cols[F].end());
        ctx->bsr_row_ptr[F + 1] = ctx->bsr_row_ptr[F] + (int)cols[F].size();
    }
    int nnzb = ctx->bsr_row_ptr[nf];
    for (int F = 0; F < nf; ++F)
        if (ctx->bsr_row_ptr[F + 1] - ctx->bsr_row_ptr[F] > 16) return fail(HDG_ERR_UNSUPPORTED);  // matvec row cache
    ctx->bsr_col.resize(nnzb);
    ctx->bsr_val_off.assign(nnzb + 1, 0);
    for (int F = 0; F < nf; ++F)
        for (size_t k = 0; k < cols[F].size(); ++k) {
            int kk = ctx->bsr_row_ptr[F] + (int)k, G = cols[F][k];
            ctx->bsr_col[kk] = G;
            // every block starts on a 128-byte line (16 doubles): the matvec streams whole lines
            const int64_t sz = (int64_t)trace_size(ctx->face_p[F]) * trace_size(ctx->face_p[G]);
            ctx->bsr_val_off[kk + 1] = (ctx->bsr_val_off[kk] + sz + 15) / 16 * 16;
        }
    auto blk_index = [&](int F, int G) {
        auto b = ctx->bsr_col.begin() + ctx->bsr_row_ptr[F], en = ctx->bsr_col.begin() + ctx->bsr_row_ptr[F + 1];
        return (int)(std::lower_bound(b, en, G) - ctx->bsr_col.begin());
    };
    std::vector<std::vector<int>> contrib(nnzb);
    std::vector<int> asm_blk(36 * ne);
    for (int e = 0; e < ne; ++e)
        for (int a = 0; a < 6; ++a)
            for (int b = 0; b < 6; ++b) {
                int k = blk_index(ctx->elem_face[6 * e + a], ctx->elem_face[6 * e + b]);
                contrib[k].insert(contrib[k].end(), {e, a, b});
                asm_blk[36 * e + 6 * a + b] = k;
            }
    std::vector<int> blk_src_ptr(nnzb + 1, 0), blk_src;
    for (int k = 0; k < nnzb; ++k) {
        blk_src_ptr[k + 1] = blk_src_ptr[k] + (int)contrib[k].size() / 3;
        blk_src.insert(blk_src.end(), contrib[k].begin(), contrib[k].end());
    }
    std::vector<int> face_src_ptr(nf + 1, 0), face_src;
    {
        std::vector<std::vector<int>> fs(nf);
        for (int e = 0; e < ne; ++e)
            for (int a = 0; a < 6; ++a) fs[ctx->elem_face[6 * e + a]].insert(fs[ctx->elem_face[6 * e + a]].end(), {e, a});
        for (int F = 0; F < nf; ++F) {
            face_src_ptr[F + 1] = face_src_ptr[F] + (int)fs[F].size() / 2;
            face_src.insert(face_src.end(), fs[F].begin(), fs[F].end());
        }
    }
    // ---- vertex classes for the artificial-viscosity smoothing: the corners of
    // the two sides of every two-sided face (periodic pairs included) are the
    // same vertices; matching corners have the same tangential position
    std::vector<int> av_corner(8 * ne), av_src_ptr, av_src;
    int n_vclass = 0;
    {
        std::vector<int> parent(m->n_vert);
        for (int v = 0; v < m->n_vert; ++v) parent[v] = v;
        std::function<int(int)> root = [&](int v) {
            while (parent[v] != v) v = parent[v] = parent[parent[v]];
            return v;
        };
        for (int F = 0; F < nf; ++F) {
            const int e0 = ctx->face_elem[4 * F], l0 = ctx->face_elem[4 * F + 1];
            const int e1 = ctx->face_elem[4 * F + 2], l1 = ctx->face_elem[4 * F + 3];
            if (e1 < 0) continue;
            const int d = l0 / 2;
            for (int c = 0; c < 8; ++c) {
                if (((c >> d) & 1) != (l0 & 1)) continue;
                const int c1 = (c & ~(1 << d)) | ((l1 & 1) << d);
                const int a = root(m->elem_vert[8 * e0 + c]), b = root(m->elem_vert[8 * e1 + c1]);
                if (a != b) parent[std::max(a, b)] = std::min(a, b);
            }
        }
        std::vector<int> id(m->n_vert, -1);
        for (int e = 0; e < ne; ++e)
            for (int c = 0; c < 8; ++c) {
                const int r = root(m->elem_vert[8 * e + c]);
                if (id[r] < 0) id[r] = n_vclass++;
                av_corner[8 * e + c] = id[r];
            }
        std::vector<std::vector<int>> src(n_vclass);
        for (int e = 0; e < ne; ++e)
            for (int c = 0; c < 8; ++c) src[av_corner[8 * e + c]].push_back(e);
        av_src_ptr.assign(n_vclass + 1, 0);
        for (int k = 0; k < n_vclass; ++k) {
            av_src_ptr[k + 1] = av_src_ptr[k] + (int)src[k].size();
            av_src.insert(av_src.end(), src[k].begin(), src[k].end());
        }
    }
    ctx->n_vclass = n_vclass;
    // ---- upload (first HIP call: everything above is host-side validation and set-up)
    if (hipGetDevice(&ctx->device) != hipSuccess) return fail(HDG_ERR_DEVICE);
    if (hdg::asm_scratch_init(ctx->device) != 0) return fail(HDG_ERR_DEVICE);
    DevMesh &dm = ctx->dm;
    dm.n_elem = ne;
    dm.n_face = nf;
    int st = HDG_OK;
#define UP(vec, field) do { if ((st = upload(ctx, vec, &dm.field)) != HDG_OK) return fail(st); } while (0)
    UP(ctx->elem_p, elem_p);
    UP(ctx->face_p, face_p);
    UP(ctx->elem_face, elem_face);
    UP(ctx->face_bc, face_bc);
    UP(ctx->toff, toff);
    UP(ctx->node_off, node_off);
    UP(ctx->face_off, face_off);
    UP(ctx->E_off, E_off);
    UP(ctx->SK_off, SK_off);
    UP(ctx->asm_off, asm_off);
    UP(ctx->qp_off, qp_off);
    UP(ctx->asmsys_off, asmsys_off);
    UP(ctx->tloc_off, tloc_off);
    UP(ctx->m32_off, m32_off);
    UP(ctx->x_off, x_off);
    UP(ctx->vgeo_off, vgeo_off);
    UP(ctx->fgeo_off, fgeo_off);
    UP(vgeo, vgeo);
    UP(fgeo, fgeo);
    UP(tbl, tbl);
    UP(ctx->bsr_row_ptr, bsr_row_ptr);
    UP(ctx->bsr_col, bsr_col);
    UP(ctx->bsr_val_off, bsr_val_off);
    UP(blk_src_ptr, blk_src_ptr);
    UP(blk_src, blk_src);
    UP(face_src_ptr, face_src_ptr);
    UP(face_src, face_src);
    UP(asm_blk, asm_blk);
    UP(av_corner, av_corner);
    UP(av_src_ptr, av_src_ptr);
    UP(av_src, av_src);
    dm.n_vclass = n_vclass;
#undef UP
    ctx->bsr_row_ptr64.assign(ctx->bsr_row_ptr.begin(), ctx->bsr_row_ptr.end());
    ctx->bsr_col64.assign(ctx->bsr_col.begin(), ctx->bsr_col.end());
    *out = ctx;
    return HDG_OK;
}

int64_t hdg_layout_length(const hdg_ctx *ctx, int kind) {
    if (!ctx) return -1;
    switch (kind) {
        case HDG_LAYOUT_NODE_OFF: case HDG_LAYOUT_E_OFF: case HDG_LAYOUT_SK_OFF: case HDG_LAYOUT_ASM_OFF:
        case HDG_LAYOUT_X_OFF:
            return ctx->n_elem + 1;
        case HDG_LAYOUT_FACE_OFF: case HDG_LAYOUT_BSR_ROW_PTR: return ctx->n_face + 1;
        case HDG_LAYOUT_BSR_COL: return (int64_t)ctx->bsr_col.size();
        case HDG_LAYOUT_BSR_VAL_OFF: return (int64_t)ctx->bsr_val_off.size();
        case HDG_LAYOUT_ELEM_N: case HDG_LAYOUT_ELEM_F: return ctx->n_elem;
        default: return -1;
    }
}

int hdg_layout(const hdg_ctx *ctx, int kind, int64_t *dst, int64_t capacity) {
    if (!ctx || !dst) return HDG_ERR_INVALID_ARGUMENT;
    int64_t len = hdg_layout_length(ctx, kind);
    if (len < 0 || capacity < len) return HDG_ERR_INVALID_ARGUMENT;
    const std::vector<int64_t> *v = nullptr;
    switch (kind) {
        case HDG_LAYOUT_NODE_OFF: v = &ctx->node_off; break;
        case HDG_LAYOUT_FACE_OFF: v = &ctx->face_off; break;
        case HDG_LAYOUT_E_OFF: v = &ctx->E_off; break;
        case HDG_LAYOUT_SK_OFF: v = &ctx->SK_off; break;
        case HDG_LAYOUT_ASM_OFF: v = &ctx->asm_off; break;
        case HDG_LAYOUT_X_OFF: v = &ctx->x_off; break;
        case HDG_LAYOUT_BSR_ROW_PTR: v = &ctx->bsr_row_ptr64; break;
        case HDG_LAYOUT_BSR_COL: v = &ctx->bsr_col64; break;
        case HDG_LAYOUT_BSR_VAL_OFF: v = &ctx->bsr_val_off; break;
        case HDG_LAYOUT_ELEM_N:
            for (int e = 0; e < ctx->n_elem; ++e) dst[e] = ctx->elem_n[e];
            return HDG_OK;
        case HDG_LAYOUT_ELEM_F:
            for (int e = 0; e < ctx->n_elem; ++e) dst[e] = ctx->elem_f[e];
            return HDG_OK;
    }
    std::copy(v->begin(), v->end(), dst);
    return HDG_OK;
}

int hdg_bsr_pattern(const hdg_ctx *ctx, int *nnzb, const int **row_ptr_dev, const int **col_dev) {
    if (!ctx) return HDG_ERR_INVALID_ARGUMENT;
    if (nnzb) *nnzb = (int)ctx->bsr_col.size();
    if (row_ptr_dev) *row_ptr_dev = ctx->dm.bsr_row_ptr;
    if (col_dev) *col_dev = ctx->dm.bsr_col;
    return HDG_OK;
}

static bool chunk_ok(const hdg_ctx *ctx, int e0, int ne) {
    return ctx && e0 >= 0 && ne >= 1 && (int64_t)e0 + ne <= ctx->n_elem;
}

static size_t round256(size_t b) { return (b + 255) / 256 * 256; }

int hdg_workspace_size(const hdg_ctx *ctx, int op, int prec, int e0, int ne, size_t *bytes) {
    if (!ctx || !bytes || (prec != HDG_FP64 && prec != HDG_MIXED && !(op == 1 && prec == HDG_MIXED_FAST)))
        return HDG_ERR_INVALID_ARGUMENT;
    switch (op) {
        case 0:  // hdg_local_residual_jacobian
            if (!chunk_ok(ctx, e0, ne)) return HDG_ERR_INVALID_ARGUMENT;
            *bytes = round256(sizeof(double) * (size_t)(ctx->qp_off[e0 + ne] - ctx->qp_off[e0]));
            return HDG_OK;
        case 1:  // hdg_condense
            if (!chunk_ok(ctx, e0, ne)) return HDG_ERR_INVALID_ARGUMENT;
            *bytes = (prec == HDG_FP64)    ? round256(hdg::bordered_lu_work(ctx, ne))
                     : (prec == HDG_MIXED) ? hdg::condense_mixed_work_bytes(ctx, e0, ne)
                                           : hdg::condense_fast_work_bytes(ctx, e0, ne);
            return HDG_OK;
        case 2: *bytes = hdg::asm_setup_work_bytes(ctx, prec); return HDG_OK;
        case 3: *bytes = hdg::asm_apply_work_bytes(ctx); return HDG_OK;
        case 4:
            if (ne < 1 || ne > 200) return HDG_ERR_INVALID_ARGUMENT;
            *bytes = hdg::gmres_work_bytes(ctx, ne);
            return HDG_OK;
        case 5:
            if (ne < 1 || ne > HDG_RB_MAX) return HDG_ERR_INVALID_ARGUMENT;
            *bytes = hdg::rb_work_bytes(ctx, ne);
            return HDG_OK;
        case 6: *bytes = hdg::resid_work_bytes(ctx); return HDG_OK;
        case 7: *bytes = hdg::av_work_bytes(ctx); return HDG_OK;
        default: return HDG_ERR_INVALID_ARGUMENT;
    }
}

static int dev_status(int hip_err) { return hip_err == 0 ? HDG_OK : HDG_ERR_DEVICE; }
// boundary types that read the prescribed state Ub (prescribed state, isothermal wall)
static bool needs_ub(int bc) { return bc == 1 || bc == 3; }

int hdg_local_residual_jacobian(hdg_ctx *ctx, int e0, int ne, const double *Q, const double *U,
                                const double *Un, const double *Uhat, const double *nu, const double *Ub,
                                double *E, void *work, size_t work_bytes, void *stream) {
    if (!chunk_ok(ctx, e0, ne) || !Q || !U || !Un || !Uhat || !nu || !E || !work) return HDG_ERR_INVALID_ARGUMENT;
    for (int e = e0; e < e0 + ne; ++e)
        for (int lf = 0; lf < 6; ++lf)
            if (needs_ub(ctx->face_bc[ctx->elem_face[6 * e + lf]]) && !Ub) return HDG_ERR_INVALID_ARGUMENT;
    size_t need;
    hdg_workspace_size(ctx, 0, HDG_FP64, e0, ne, &need);
    if (work_bytes < need) return HDG_ERR_WORKSPACE;
    return dev_status(hdg::launch_element_system(ctx, e0, ne, Q, U, Un, Uhat, nu, Ub, E, (double *)work,
                                                 (hipStream_t)stream));
}

int hdg_condense(hdg_ctx *ctx, int prec, int refine_steps, int e0, int ne, double *E, double *SK, int *info,
                 void *work, size_t work_bytes, void *stream) {
    if (!chunk_ok(ctx, e0, ne) || !E || !SK || !info) return HDG_ERR_INVALID_ARGUMENT;
    if (prec != HDG_FP64 && prec != HDG_MIXED && prec != HDG_MIXED_FAST) return HDG_ERR_INVALID_ARGUMENT;
    if (prec == HDG_MIXED && (refine_steps < 1 || refine_steps > 8)) return HDG_ERR_INVALID_ARGUMENT;
    size_t need;
    hdg_workspace_size(ctx, 1, prec, e0, ne, &need);
    if (!work || work_bytes < need) return HDG_ERR_WORKSPACE;
    if (prec == HDG_FP64)
        return dev_status(hdg::launch_condense_fp64(ctx, e0, ne, E, SK, info, work, (hipStream_t)stream));
    if (prec == HDG_MIXED_FAST)
        return dev_status(hdg::launch_condense_fast(ctx, e0, ne, E, SK, info, work, (hipStream_t)stream));
    return dev_status(hdg::launch_condense_mixed(ctx, e0, ne, refine_steps, E, SK, info, work, (hipStream_t)stream));
}

int hdg_assemble_trace(hdg_ctx *ctx, const double *SK, double *S_bsr, double *g, void *stream) {
    if (!ctx || !SK || !S_bsr || !g) return HDG_ERR_INVALID_ARGUMENT;
    return dev_status(hdg::launch_assemble(ctx, SK, S_bsr, g, (hipStream_t)stream));
}

int hdg_peak_mfma(int fp_bits, int n_wg, int iters, double one, void *sink, void *stream) {
    if ((fp_bits != 64 && fp_bits != 32) || n_wg < 1 || n_wg > (1 << 20) || iters < 1 || !sink)
        return HDG_ERR_INVALID_ARGUMENT;
    return dev_status(hdg::launch_peak_mfma(fp_bits, n_wg, iters, one, sink, (hipStream_t)stream));
}

int hdg_peak_read(const void *src, size_t bytes, unsigned *sink, void *stream) {
    if (!src || !sink || bytes == 0 || bytes % 16 || (uintptr_t)src % 16) return HDG_ERR_INVALID_ARGUMENT;
    return dev_status(hdg::launch_peak_read(src, bytes, sink, (hipStream_t)stream));
}

int hdg_peak_copy(const void *src, void *dst, size_t bytes, void *stream) {
    const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
    if (!src || !dst || bytes == 0 || bytes % 16 || a % 16 || b % 16 || (a < b + bytes && b < a + bytes))
        return HDG_ERR_INVALID_ARGUMENT;
    return dev_status(hdg::launch_peak_copy(src, dst, bytes, (hipStream_t)stream));
}

int hdg_face_matvec(hdg_ctx *ctx, const double *S_bsr, const double *x, double *y, void *stream) {
    if (!ctx || !S_bsr || !x || !y || x == y) return HDG_ERR_INVALID_ARGUMENT;
    return dev_status(hdg::launch_matvec(ctx, S_bsr, x, y, (hipStream_t)stream));
}

int hdg_asm_setup(hdg_ctx *ctx, int prec, const double *S_bsr, void *Sinv, int *info, void *work,
                  size_t work_bytes, void *stream) {
    if (!ctx || !S_bsr || !Sinv || !info || (prec != HDG_FP64 && prec != HDG_MIXED)) return HDG_ERR_INVALID_ARGUMENT;
    if (ctx->repeated_face) return HDG_ERR_UNSUPPORTED;
    if (work_bytes < hdg::asm_setup_work_bytes(ctx, prec) || !work) return HDG_ERR_WORKSPACE;
    return dev_status(hdg::launch_asm_setup(ctx, prec, S_bsr, Sinv, info, work, (hipStream_t)stream));
}

int hdg_asm_block_apply(hdg_ctx *ctx, int prec, const void *Sinv, const double *r, double *z, void *work,
                        size_t work_bytes, void *stream) {
    if (!ctx || !Sinv || !r || !z || r == z || (prec != HDG_FP64 && prec != HDG_MIXED)) return HDG_ERR_INVALID_ARGUMENT;
    if (work_bytes < hdg::asm_apply_work_bytes(ctx) || !work) return HDG_ERR_WORKSPACE;
    return dev_status(hdg::launch_asm_apply(ctx, prec, Sinv, r, z, work, (hipStream_t)stream));
}

int hdg_asm_block_apply_noalloc(hdg_ctx *ctx, int prec, const void *Sinv, const double *r, double *z,
                                void *stream) {
    if (!ctx || !Sinv || !r || !z || r == z || (prec != HDG_FP64 && prec != HDG_MIXED)) return HDG_ERR_INVALID_ARGUMENT;
    if ((size_t)ctx->tloc_off[ctx->n_elem] > hdg::kAsmScratchDoubles) return HDG_ERR_WORKSPACE;
    return dev_status(hdg::launch_asm_apply_noalloc(ctx, prec, Sinv, r, z, (hipStream_t)stream));
}

int hdg_gmres(hdg_ctx *ctx, int prec, const double *S_bsr, const void *Sinv, const double *g, int m,
              double *dUhat, double *res_hist, void *work, size_t work_bytes, void *stream) {
    if (!ctx || !S_bsr || !Sinv || !g || !dUhat || !res_hist || m < 1 || m > 200 ||
        (prec != HDG_FP64 && prec != HDG_MIXED))
        return HDG_ERR_INVALID_ARGUMENT;
    if (work_bytes < hdg::gmres_work_bytes(ctx, m) || !work) return HDG_ERR_WORKSPACE;
    return dev_status(hdg::launch_gmres(ctx, prec, S_bsr, Sinv, g, nullptr, m, dUhat, res_hist, work,
                                        (hipStream_t)stream));
}

int hdg_gmres_x0(hdg_ctx *ctx, int prec, const double *S_bsr, const void *Sinv, const double *g, const double *x0,
                 int m, double *dUhat, double *res_hist, void *work, size_t work_bytes, void *stream) {
    if (!ctx || !S_bsr || !Sinv || !g || !x0 || !dUhat || !res_hist || m < 1 || m > 200 ||
        (prec != HDG_FP64 && prec != HDG_MIXED))
        return HDG_ERR_INVALID_ARGUMENT;
    if (work_bytes < hdg::gmres_work_bytes(ctx, m) || !work) return HDG_ERR_WORKSPACE;
    return dev_status(hdg::launch_gmres(ctx, prec, S_bsr, Sinv, g, x0, m, dUhat, res_hist, work,
                                        (hipStream_t)stream));
}

int hdg_rb_guess(hdg_ctx *ctx, int nb, const double *W, const double *Z, const double *g, double *x0, void *work,
                 size_t work_bytes, void *stream) {
    if (!ctx || !g || !x0 || nb < 0 || nb > HDG_RB_MAX || (nb > 0 && (!W || !Z))) return HDG_ERR_INVALID_ARGUMENT;
    if (nb > 0 && (!work || work_bytes < hdg::rb_work_bytes(ctx, nb))) return HDG_ERR_WORKSPACE;
    return dev_status(hdg::launch_rb_guess(ctx, nb, W, Z, g, x0, work, (hipStream_t)stream));
}

int hdg_rb_insert(hdg_ctx *ctx, const double *S_bsr, const double *w_new, int nb_max, int *count, int *head,
                  double *W, double *Z, void *stream) {
    if (!ctx || !S_bsr || !w_new || !count || !head || !W || !Z || nb_max < 1 || nb_max > HDG_RB_MAX)
        return HDG_ERR_INVALID_ARGUMENT;
    if (*count < 0 || *count > nb_max || *head < 0 || *head >= nb_max) return HDG_ERR_INVALID_ARGUMENT;
    const int rc = hdg::launch_rb_insert(ctx, S_bsr, w_new, *head, W, Z, (hipStream_t)stream);
    if (rc) return HDG_ERR_DEVICE;
    *head = (*head + 1) % nb_max;
    *count = std::min(*count + 1, nb_max);
    return HDG_OK;
}

int hdg_state_update(hdg_ctx *ctx, double alpha, const double *dQU, const double *dUhat, double *Q, double *U,
                     double *Uhat, void *stream) {
    if (!ctx || !dQU || !dUhat || !Q || !U || !Uhat || !std::isfinite(alpha)) return HDG_ERR_INVALID_ARGUMENT;
    return dev_status(hdg::launch_state_update(ctx, alpha, dQU, dUhat, Q, U, Uhat, (hipStream_t)stream));
}

int hdg_state_admissible(hdg_ctx *ctx, double alpha, const double *U, const double *dQU, int *flag, void *stream) {
    if (!ctx || !U || !dQU || !flag || !std::isfinite(alpha)) return HDG_ERR_INVALID_ARGUMENT;
    return dev_status(hdg::launch_admissible(ctx, alpha, U, dQU, flag, (hipStream_t)stream));
}

int hdg_lincomb(hdg_ctx *ctx, int k, const double *const *v, const double *coef, double *out, int64_t n,
                void *stream) {
    if (!ctx || k < 1 || k > 8 || !v || !coef || !out || n < 0) return HDG_ERR_INVALID_ARGUMENT;
    for (int i = 0; i < k; ++i)
        if (!v[i] || !std::isfinite(coef[i])) return HDG_ERR_INVALID_ARGUMENT;
    if (n == 0) return HDG_OK;
    return dev_status(hdg::launch_lincomb(k, v, coef, out, n, (hipStream_t)stream));
}

int hdg_residual_gather(hdg_ctx *ctx, int e0, int ne, const double *E, void *work, size_t work_bytes, void *stream) {
    if (!chunk_ok(ctx, e0, ne) || !E) return HDG_ERR_INVALID_ARGUMENT;
    if (!work || work_bytes < hdg::resid_work_bytes(ctx)) return HDG_ERR_WORKSPACE;
    return dev_status(hdg::launch_resid_elem(ctx, e0, ne, E, work, (hipStream_t)stream));
}

int hdg_av_field(hdg_ctx *ctx, const hdg_av_params *ap, const double *U, const double *Q, double *nu_raw,
                 double *nu, void *work, size_t work_bytes, void *stream) {
    if (!ctx || !ap || !U || !Q || !nu) return HDG_ERR_INVALID_ARGUMENT;
    if (!(ap->c_av >= 0.0) || !(ap->h_m > 0.0) || !(ap->eps > 0.0) || !(ap->s_max > 0.0) ||
        !(ap->rho_min > 0.0) || !(ap->p_min > 0.0) || ap->smooth_iters < 0 || ap->smooth_iters > 64)
        return HDG_ERR_INVALID_ARGUMENT;
    if (!work || work_bytes < hdg::av_work_bytes(ctx)) return HDG_ERR_WORKSPACE;
    const hdg::AvParams p{ap->c_av, ap->h_m, ap->eps, ap->s_max, ap->rho_min, ap->p_min, ap->smooth_iters};
    return dev_status(hdg::launch_av_field(ctx, p, U, Q, nu_raw, nu, work, (hipStream_t)stream));
}

int hdg_residual_norm(hdg_ctx *ctx, void *work, size_t work_bytes, double *norms, void *stream) {
    if (!ctx || !norms) return HDG_ERR_INVALID_ARGUMENT;
    if (!work || work_bytes < hdg::resid_work_bytes(ctx)) return HDG_ERR_WORKSPACE;
    return dev_status(hdg::launch_resid_norm(ctx, work, norms, (hipStream_t)stream));
}

int hdg_recover_interior(hdg_ctx *ctx, int prec, int e0, int ne, const double *E, const double *dUhat,
                         double *dQU, void *stream) {
    if (!chunk_ok(ctx, e0, ne) || !E || !dUhat || !dQU ||
        (prec != HDG_FP64 && prec != HDG_MIXED && prec != HDG_MIXED_FAST))
        return HDG_ERR_INVALID_ARGUMENT;
    if (prec == HDG_MIXED_FAST) prec = HDG_FP64;  // E holds U and L^{-1} P [B | R_qu] in either case
    return dev_status(hdg::launch_recover(ctx, prec, e0, ne, E, dUhat, dQU, (hipStream_t)stream));
}

int hdg_store_x(hdg_ctx *ctx, int e0, int ne, const double *E, double *X, void *stream) {
    if (!chunk_ok(ctx, e0, ne) || !E || !X) return HDG_ERR_INVALID_ARGUMENT;
    return dev_status(hdg::launch_store_x(ctx, e0, ne, E, X, (hipStream_t)stream));
}

int hdg_recover_interior_x(hdg_ctx *ctx, int e0, int ne, const double *X, const double *dUhat, double *dQU,
                           void *stream) {
    if (!chunk_ok(ctx, e0, ne) || !X || !dUhat || !dQU) return HDG_ERR_INVALID_ARGUMENT;
    return dev_status(hdg::launch_recover_x(ctx, e0, ne, X, dUhat, dQU, (hipStream_t)stream));
}

// ------------------------------------------------------ the whole step
static int newton_check(hdg_ctx *ctx, const hdg_newton_args *a) {
    if (!ctx || !a) return HDG_ERR_INVALID_ARGUMENT;
    if ((a->prec != HDG_FP64 && a->prec != HDG_MIXED && a->prec != HDG_MIXED_FAST) ||
        (a->asm_prec != HDG_FP64 && a->asm_prec != HDG_MIXED))
        return HDG_ERR_INVALID_ARGUMENT;
    if (a->prec == HDG_MIXED && (a->refine_steps < 1 || a->refine_steps > 8)) return HDG_ERR_INVALID_ARGUMENT;
    if (a->gmres_m < 1 || a->gmres_m > 200) return HDG_ERR_INVALID_ARGUMENT;
    if (a->n_chunks < 1 || !a->chunk_e0 || !a->chunk_ne) return HDG_ERR_INVALID_ARGUMENT;
    if (!a->Q || !a->U || !a->Un || !a->Uhat || !a->nu || !a->E || !a->qp_work || !a->cond_work || !a->SK ||
        !a->info || !a->S_bsr || !a->g || !a->Sinv || !a->asm_info || !a->asm_work || !a->gmres_work ||
        !a->dUhat || !a->res_hist || !a->dQU)
        return HDG_ERR_INVALID_ARGUMENT;
    // every element in exactly one chunk
    std::vector<char> seen(ctx->n_elem, 0);
    for (int k = 0; k < a->n_chunks; ++k) {
        const int e0 = a->chunk_e0[k], ne = a->chunk_ne[k];
        if (!chunk_ok(ctx, e0, ne)) return HDG_ERR_INVALID_ARGUMENT;
        for (int e = e0; e < e0 + ne; ++e) {
            if (seen[e]) return HDG_ERR_INVALID_ARGUMENT;
            seen[e] = 1;
        }
        size_t need;
        hdg_workspace_size(ctx, 0, HDG_FP64, e0, ne, &need);
        if (a->qp_work_bytes < need) return HDG_ERR_WORKSPACE;
        hdg_workspace_size(ctx, 1, a->prec, e0, ne, &need);
        if (a->cond_work_bytes < need) return HDG_ERR_WORKSPACE;
    }
    for (int e = 0; e < ctx->n_elem; ++e)
        if (!seen[e]) return HDG_ERR_INVALID_ARGUMENT;
    if (!a->Ub)
        for (int F = 0; F < ctx->n_face; ++F)
            if (needs_ub(ctx->face_bc[F])) return HDG_ERR_INVALID_ARGUMENT;
    if (ctx->repeated_face) return HDG_ERR_UNSUPPORTED;
    if (a->asm_work_bytes < hdg::asm_setup_work_bytes(ctx, a->asm_prec)) return HDG_ERR_WORKSPACE;
    if (a->gmres_work_bytes < hdg::gmres_work_bytes(ctx, a->gmres_m)) return HDG_ERR_WORKSPACE;
    return HDG_OK;
}

// The step's calls in order (arguments already checked).
static int newton_enqueue(hdg_ctx *ctx, const hdg_newton_args *a, void *stream) {
    int rc;
    auto Ek = [&](int e0) { return a->E + ctx->E_off[e0]; };
    for (int k = 0; k < a->n_chunks; ++k) {
        const int e0 = a->chunk_e0[k], ne = a->chunk_ne[k];
        if ((rc = hdg_local_residual_jacobian(ctx, e0, ne, a->Q, a->U, a->Un, a->Uhat, a->nu, a->Ub, Ek(e0),
                                              a->qp_work, a->qp_work_bytes, stream)))
            return rc;
        if ((rc = hdg_condense(ctx, a->prec, a->refine_steps, e0, ne, Ek(e0), a->SK, a->info, a->cond_work,
                               a->cond_work_bytes, stream)))
            return rc;
    }
    if ((rc = hdg_assemble_trace(ctx, a->SK, a->S_bsr, a->g, stream))) return rc;
    if ((rc = hdg_asm_setup(ctx, a->asm_prec, a->S_bsr, a->Sinv, a->asm_info, a->asm_work, a->asm_work_bytes,
                            stream)))
        return rc;
    if ((rc = hdg_gmres(ctx, a->asm_prec, a->S_bsr, a->Sinv, a->g, a->gmres_m, a->dUhat, a->res_hist,
                        a->gmres_work, a->gmres_work_bytes, stream)))
        return rc;
    // every system is resident: one recovery launch over all elements keeps several
    // workgroups per CU busy on the sequential block steps of the back substitution
    return hdg_recover_interior(ctx, a->prec, 0, ctx->n_elem, a->E, a->dUhat, a->dQU, stream);
}

int hdg_set_update_tile(hdg_ctx *ctx, int n, int tile_rows) {
    if (!ctx || n < 0 || (tile_rows != 128 && tile_rows != 256)) return HDG_ERR_INVALID_ARGUMENT;
    ctx->update_tile[n] = tile_rows;
    return HDG_OK;
}

int hdg_get_update_tile(const hdg_ctx *ctx, int n) {
    if (!ctx || n < 0) return HDG_ERR_INVALID_ARGUMENT;
    auto it = ctx->update_tile.find(n);
    if (it != ctx->update_tile.end()) return it->second;
    it = ctx->update_tile.find(0);
    return it != ctx->update_tile.end() ? it->second : 128;
}

int hdg_newton_step(hdg_ctx *ctx, const hdg_newton_args *args, void *stream) {
    const int rc = newton_check(ctx, args);
    if (rc) return rc;
    return newton_enqueue(ctx, args, stream);
}

}  // extern "C"

struct hdg_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" {

void hdg_graph_destroy(hdg_graph *gr) {
    if (!gr) return;
    if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
    if (gr->graph) (void)hipGraphDestroy(gr->graph);
    delete gr;
}

int hdg_graph_capture_newton(hdg_ctx *ctx, const hdg_newton_args *args, hdg_graph **out, void *stream) {
    if (!out || !stream) return HDG_ERR_INVALID_ARGUMENT;
    *out = nullptr;
    int rc = newton_check(ctx, args);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    // one eager run: every kernel's code object is loaded before the capture
    if ((rc = newton_enqueue(ctx, args, stream))) return rc;
    if (hipStreamSynchronize(s) != hipSuccess) return HDG_ERR_DEVICE;
    hdg_graph *gr = new (std::nothrow) hdg_graph();
    if (!gr) return HDG_ERR_OUT_OF_MEMORY;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        delete gr;
        return HDG_ERR_DEVICE;
    }
    rc = newton_enqueue(ctx, args, stream);
    const hipError_t end = hipStreamEndCapture(s, &gr->graph);
    if (rc || end != hipSuccess || !gr->graph) {
        hdg_graph_destroy(gr);
        return rc ? rc : HDG_ERR_DEVICE;
    }
    if (hipGraphInstantiate(&gr->exec, gr->graph, nullptr, nullptr, 0) != hipSuccess) {
        hdg_graph_destroy(gr);
        return HDG_ERR_DEVICE;
    }
    *out = gr;
    return HDG_OK;
}

int hdg_graph_launch(hdg_graph *gr, void *stream) {
    if (!gr || !gr->exec) return HDG_ERR_INVALID_ARGUMENT;
    return hipGraphLaunch(gr->exec, (hipStream_t)stream) == hipSuccess ? HDG_OK : HDG_ERR_DEVICE;
}

}  // extern "C"
