/*
 * hdgref.c -- plain, slow FP64 CPU oracle for the HDG element-local hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; it shares no code, header or table with the HIP path.
 * Only tests, the smoke check and the benchmark's CPU-baseline leg use it.
 *
 * What it computes (Welter, Collin, Nguyen, Peraire: HDG solver for DNS of
 * compressible flows on GPUs):
 *   - conservative compressible Navier-Stokes fluxes: inviscid flux
 *     (eq. convective-flux), ideal gas (eq. ideal-gas), viscous flux with
 *     Stokes stress and Fourier heat flux (eqs. viscous-flux, stress-heat,
 *     thermal-conductivity), nondimensional Sutherland viscosity
 *     (eq. tgv-sutherland), artificial-viscosity flux nu * grad u (eq. av-total);
 *   - the HDG weak form (eqs. hdg-grad, hdg-cons, hdg-trace) with the
 *     numerical flux of eq. num-flux-hdg, the DIRK stage mass term of
 *     eq. fully-discrete-local, on tensor-product hexahedra;
 *   - the element Newton block of eq. newton-local-block (A, B), the trace
 *     equation's linearisation (C, D), all by forward-mode dual numbers;
 *   - static condensation, eqs. local-elimination and schur-trace, by a
 *     textbook LU with partial pivoting.
 *
 * Layout written (the library's documented element-system layout):
 *   E is column-major with leading dimension n+f, n = 20 N_p, f = sum of the
 *   element's 6 face trace sizes 5 (p_F+1)^2, and n+f+1 columns:
 *       [ A  B  R_qu ]   rows 0..n-1     (interior equations)
 *       [ C  D  R_uh ]   rows n..n+f-1   (this element's trace equations)
 *   interior index = field * N_p + node, field = 3c+j for q_{c,j}, 15+c for u_c;
 *   trace index    = toff[lf] + c * N_fp(lf) + a, faces in -x,+x,-y,+y,-z,+z order.
 *
 * Build: gcc -O2 -shared -fPIC -o liboracle.so hdgref.c -lm
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* 1-D Legendre polynomials, Gauss and Gauss-Lobatto rules, Lagrange   */
/* ------------------------------------------------------------------ */
static void legendre_eval(int n, double x, double *P, double *dP)
{
    /* Bonnet recurrence; derivative from (1-x^2) P_n' = n (P_{n-1} - x P_n). */
    double p0 = 1.0, p1 = x;
    if (n == 0) { *P = 1.0; *dP = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1; p1 = p2;
    }
    *P = p1;
    if (fabs(x) < 1.0) *dP = n * (p0 - x * p1) / (1.0 - x * x);
    else *dP = 0.5 * n * (n + 1.0) * (x > 0 ? 1.0 : ((n % 2) ? 1.0 : -1.0));
}

/* Gauss-Legendre: roots of P_nq by Newton, weights 2 / ((1-x^2) P'(x)^2). */
void hdgref_gauss(int nq, double *x, double *w)
{
    for (int i = 0; i < nq; ++i) {
        double xi = -cos(M_PI * (i + 0.75) / (nq + 0.5));
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre_eval(nq, xi, &P, &dP);
            double dx = P / dP;
            xi -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        double P, dP;
        legendre_eval(nq, xi, &P, &dP);
        x[i] = xi;
        w[i] = 2.0 / ((1.0 - xi * xi) * dP * dP);
    }
}

/* Gauss-Lobatto: -1, roots of P_p' (Newton with P'' from Legendre's ODE), +1. */
void hdgref_gll(int p, double *x)
{
    x[0] = -1.0;
    x[p] = 1.0;
    for (int i = 1; i < p; ++i) {
        double xi = -cos(M_PI * i / p);
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre_eval(p, xi, &P, &dP);
            double d2P = (2.0 * xi * dP - p * (p + 1.0) * P) / (1.0 - xi * xi);
            double dx = dP / d2P;
            xi -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        x[i] = xi;
    }
}

/* Lagrange polynomials on nodes r[0..p], value and derivative at t. */
static void lagrange(int p, const double *r, double t, double *val, double *der)
{
    for (int a = 0; a <= p; ++a) {
        double v = 1.0, d = 0.0;
        for (int b = 0; b <= p; ++b) {
            if (b == a) continue;
            double term = 1.0 / (r[a] - r[b]);
            /* d(v * (t - r_b) term) = d * (t - r_b) term + v * term */
            d = d * (t - r[b]) * term + v * term;
            v = v * (t - r[b]) * term;
        }
        val[a] = v;
        if (der) der[a] = d;
    }
}

/* ------------------------------------------------------------------ */
/* Forward-mode dual numbers, derivative slots: u 0..4, q 5..19, uhat 20..24 */
/* ------------------------------------------------------------------ */
#define ND 25
typedef struct { double v; double d[ND]; } dual;

static dual dconst(double c) { dual r; r.v = c; memset(r.d, 0, sizeof r.d); return r; }
static dual dvar(double c, int slot) { dual r = dconst(c); r.d[slot] = 1.0; return r; }
static dual dadd(dual a, dual b) { dual r; r.v = a.v + b.v; for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
static dual dsub(dual a, dual b) { dual r; r.v = a.v - b.v; for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
static dual dmul(dual a, dual b) { dual r; r.v = a.v * b.v; for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
static dual dscale(dual a, double s) { dual r; r.v = a.v * s; for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] * s; return r; }
static dual ddiv(dual a, dual b)
{
    dual r; r.v = a.v / b.v;
    for (int k = 0; k < ND; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
    return r;
}
static dual dsqrt(dual a)
{
    dual r; r.v = sqrt(a.v);
    for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] / (2.0 * r.v);
    return r;
}

typedef struct {
    double gamma, Pr, Re, Mach, tau, dt, alpha;
    int visc_law;
} params;

/*
 * Inviscid and viscous(+AV) fluxes at one point from the state w (5) and the
 * conservative-variable gradient q (15, q[3c+j] = d u_c / d x_j).
 * Nondimensional: p = (gamma-1) rho e, T = gamma (gamma-1) M^2 e, viscosity
 * mu(T)/Re, heat flux gamma mu/(Re Pr) d e/dx_j (= kappa dT/dx_j with
 * kappa = c_p mu / Pr), AV flux nu q_{c,j} added to every component.
 */
static void fluxes(const dual *w, const dual *q, double nu, const params *P,
                   dual Fc[5][3], dual Fv[5][3])
{
    dual rho = w[0], rE = w[4];
    dual v[3], m[3];
    for (int i = 0; i < 3; ++i) { m[i] = w[1 + i]; v[i] = ddiv(m[i], rho); }
    dual E = ddiv(rE, rho);
    dual ke = dscale(dadd(dadd(dmul(v[0], v[0]), dmul(v[1], v[1])), dmul(v[2], v[2])), 0.5);
    dual e = dsub(E, ke);
    dual p = dscale(dmul(rho, e), P->gamma - 1.0);
    dual mu;
    if (P->visc_law == 1) {
        dual T = dscale(e, P->gamma * (P->gamma - 1.0) * P->Mach * P->Mach);
        /* mu(T) = 1.4042 T^{3/2} / (T + 0.40417) */
        mu = ddiv(dscale(dmul(T, dsqrt(T)), 1.4042), dadd(T, dconst(0.40417)));
    } else {
        mu = dconst(1.0);
    }
    mu = dscale(mu, 1.0 / P->Re);
    dual dv[3][3], dE[3], de[3];
    for (int j = 0; j < 3; ++j) {
        for (int i = 0; i < 3; ++i)
            dv[i][j] = ddiv(dsub(q[3 * (1 + i) + j], dmul(v[i], q[j])), rho);
        dE[j] = ddiv(dsub(q[12 + j], dmul(E, q[j])), rho);
        de[j] = dE[j];
        for (int i = 0; i < 3; ++i) de[j] = dsub(de[j], dmul(v[i], dv[i][j]));
    }
    dual div = dadd(dadd(dv[0][0], dv[1][1]), dv[2][2]);
    dual tau[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            dual s = dadd(dv[i][j], dv[j][i]);
            if (i == j) s = dsub(s, dscale(div, 2.0 / 3.0));
            tau[i][j] = dmul(mu, s);
        }
    dual rEp = dadd(rE, p);
    for (int j = 0; j < 3; ++j) {
        Fc[0][j] = m[j];
        for (int i = 0; i < 3; ++i) {
            Fc[1 + i][j] = dmul(m[i], v[j]);
            if (i == j) Fc[1 + i][j] = dadd(Fc[1 + i][j], p);
        }
        Fc[4][j] = dmul(rEp, v[j]);
        Fv[0][j] = dconst(0.0);
        for (int i = 0; i < 3; ++i) Fv[1 + i][j] = tau[i][j];
        dual en = dscale(dmul(mu, de[j]), P->gamma / P->Pr);
        for (int i = 0; i < 3; ++i) en = dadd(en, dmul(v[i], tau[i][j]));
        Fv[4][j] = en;
        for (int c = 0; c < 5; ++c) Fv[c][j] = dadd(Fv[c][j], dscale(q[3 * c + j], nu));
    }
}

/* Pointwise fluxes exposed for the identity checks (values and derivative
 * slots: Fc_out/Fv_out [5][3] values, dF_out [5][3][ND]). */
void hdgref_point_flux(const double *w, const double *q, double nu, const double *prm,
                       double *Fc_out, double *Fv_out, double *dFc_out, double *dFv_out)
{
    params P = { prm[0], prm[1], prm[2], prm[3], prm[4], prm[5], prm[6], (int)prm[7] };
    dual wd[5], qd[15], Fc[5][3], Fv[5][3];
    for (int c = 0; c < 5; ++c) wd[c] = dvar(w[c], c);
    for (int m = 0; m < 15; ++m) qd[m] = dvar(q[m], 5 + m);
    fluxes(wd, qd, nu, &P, Fc, Fv);
    for (int c = 0; c < 5; ++c)
        for (int j = 0; j < 3; ++j) {
            Fc_out[3 * c + j] = Fc[c][j].v;
            Fv_out[3 * c + j] = Fv[c][j].v;
            for (int k = 0; k < 20; ++k) {
                dFc_out[(3 * c + j) * 20 + k] = Fc[c][j].d[k];
                dFv_out[(3 * c + j) * 20 + k] = Fv[c][j].d[k];
            }
        }
}

/* ------------------------------------------------------------------ */
/* Trilinear geometry                                                   */
/* ------------------------------------------------------------------ */
static void trilinear_jac(const double *X8, const double *xi, double J[3][3], double *x)
{
    /* J[i][d] = d x_i / d xi_d */
    for (int i = 0; i < 3; ++i) { x[i] = 0.0; for (int d = 0; d < 3; ++d) J[i][d] = 0.0; }
    for (int v = 0; v < 8; ++v) {
        double s[3], f[3], df[3];
        for (int d = 0; d < 3; ++d) {
            s[d] = ((v >> d) & 1) ? 1.0 : -1.0;
            f[d] = 0.5 * (1.0 + s[d] * xi[d]);
            df[d] = 0.5 * s[d];
        }
        double N = f[0] * f[1] * f[2];
        double dN[3] = { df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2] };
        for (int i = 0; i < 3; ++i) {
            x[i] += N * X8[3 * v + i];
            for (int d = 0; d < 3; ++d) J[i][d] += dN[d] * X8[3 * v + i];
        }
    }
}

/* Geometry map of order g (1: the 8 vertices, trilinear; 2: 27 nodes,
 * triquadratic), nodes in tensor order at reference coordinates equispaced on
 * [-1, 1]: x(xi) = sum_abc X_abc l_a(xi_0) l_b(xi_1) l_c(xi_2) with the Lagrange
 * polynomials of those coordinates (the curved high-order map of section 2.2). */
static void geom_jac(int g, const double *Xg, const double *xi, double J[3][3], double *x)
{
    if (g == 1) { trilinear_jac(Xg, xi, J, x); return; }
    double r[3] = { -1.0, 0.0, 1.0 }, l[3][3], dl[3][3];
    for (int d = 0; d < 3; ++d) lagrange(2, r, xi[d], l[d], dl[d]);
    for (int i = 0; i < 3; ++i) { x[i] = 0.0; for (int d = 0; d < 3; ++d) J[i][d] = 0.0; }
    for (int c = 0; c < 3; ++c)
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a) {
                const double *X = Xg + 3 * (a + 3 * (b + 3 * c));
                double N = l[0][a] * l[1][b] * l[2][c];
                double dN[3] = { dl[0][a] * l[1][b] * l[2][c], l[0][a] * dl[1][b] * l[2][c],
                                 l[0][a] * l[1][b] * dl[2][c] };
                for (int i = 0; i < 3; ++i) {
                    x[i] += N * X[i];
                    for (int d = 0; d < 3; ++d) J[i][d] += dN[d] * X[i];
                }
            }
}

static double inv3(double J[3][3], double G[3][3])
{
    /* G = J^{-1}: G[d][j] = d xi_d / d x_j */
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
               - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
               + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    G[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    G[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    G[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    G[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    G[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    G[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    G[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    G[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    G[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    return det;
}

/* Outward area-weighted normal of face xi_d = s (s = +-1): s * (x_a x x_b) with
 * (a, b, d) cyclic. */
static void face_normal(double J[3][3], int d, double s, double *N)
{
    int a = (d + 1) % 3, b = (d + 2) % 3;
    double ta[3] = { J[0][a], J[1][a], J[2][a] }, tb[3] = { J[0][b], J[1][b], J[2][b] };
    N[0] = s * (ta[1] * tb[2] - ta[2] * tb[1]);
    N[1] = s * (ta[2] * tb[0] - ta[0] * tb[2]);
    N[2] = s * (ta[0] * tb[1] - ta[1] * tb[0]);
}

/* ------------------------------------------------------------------ */
/* Element system: residuals (eqs. hdg-grad, hdg-cons with the DIRK mass term, */
/* hdg-trace) and their exact Jacobians, written into E.                       */
/* ------------------------------------------------------------------ */
int hdgref_trace_size(int pf) { return 5 * (pf + 1) * (pf + 1); }

/*
 * p: element degree; pf[6]: face degrees; bc[6]: boundary type of each face (0 interior
 * or periodic; 1 prescribed state, 2 extrapolated state, 3 isothermal wall, 4 adiabatic
 * wall, 5 symmetry; see the boundary residual below);
 * g, Xg: geometry order (1 or 2) and its 8 or 27 nodes (tensor order) * 3;
 * prm: gamma, Pr, Re, Mach, tau, dt, alpha, visc_law;
 * Q [15][N_p], U, Un [5][N_p], nu [N_p]; Uh, Ub: element trace order [sum_lf 5 N_fp];
 * E: (n+f) x (n+f+1) column-major, overwritten.
 */
int hdgref_element_system(int p, const int *pf, const int *bc, int g, const double *Xg, const double *prm,
                          const double *Q, const double *U, const double *Un, const double *nu,
                          const double *Uh, const double *Ub, double *E)
{
    params P = { prm[0], prm[1], prm[2], prm[3], prm[4], prm[5], prm[6], (int)prm[7] };
    const int np1 = p + 1, Np = np1 * np1 * np1, n = 20 * Np;
    int toff[7];
    toff[0] = 0;
    for (int lf = 0; lf < 6; ++lf) toff[lf + 1] = toff[lf] + hdgref_trace_size(pf[lf]);
    const int f = toff[6], ld = n + f;
#define EL(r, c) E[(size_t)(r) + (size_t)(c) * (size_t)ld]
    memset(E, 0, sizeof(double) * (size_t)ld * (size_t)(ld + 1));
    const int colR = n + f;

    double r[8], xg[8], wg[8];
    hdgref_gll(p, r);
    const int nq = p + 2;
    hdgref_gauss(nq, xg, wg);
    double *phi = malloc(sizeof(double) * Np), *dphi = malloc(sizeof(double) * Np * 3);

    /* ---------------- volume terms ---------------- */
    for (int g2 = 0; g2 < nq; ++g2)
    for (int g1 = 0; g1 < nq; ++g1)
    for (int g0 = 0; g0 < nq; ++g0) {
        double xi[3] = { xg[g0], xg[g1], xg[g2] };
        double w = wg[g0] * wg[g1] * wg[g2];
        double J[3][3], G[3][3], xx[3];
        geom_jac(g, Xg, xi, J, xx);
        double det = inv3(J, G);
        double W = w * det;
        double l[3][8], dl[3][8];
        for (int d = 0; d < 3; ++d) lagrange(p, r, xi[d], l[d], dl[d]);
        for (int i2 = 0; i2 < np1; ++i2)
        for (int i1 = 0; i1 < np1; ++i1)
        for (int i0 = 0; i0 < np1; ++i0) {
            int i = i0 + np1 * (i1 + np1 * i2);
            phi[i] = l[0][i0] * l[1][i1] * l[2][i2];
            double dr[3] = { dl[0][i0] * l[1][i1] * l[2][i2],
                             l[0][i0] * dl[1][i1] * l[2][i2],
                             l[0][i0] * l[1][i1] * dl[2][i2] };
            for (int j = 0; j < 3; ++j)
                dphi[3 * i + j] = dr[0] * G[0][j] + dr[1] * G[1][j] + dr[2] * G[2][j];
        }
        double u[5] = {0}, un[5] = {0}, q[15] = {0}, nuv = 0.0;
        for (int i = 0; i < Np; ++i) {
            for (int c = 0; c < 5; ++c) { u[c] += phi[i] * U[c * Np + i]; un[c] += phi[i] * Un[c * Np + i]; }
            for (int m = 0; m < 15; ++m) q[m] += phi[i] * Q[m * Np + i];
            nuv += phi[i] * nu[i];
        }
        dual ud[5], qd[15], Fc[5][3], Fv[5][3];
        for (int c = 0; c < 5; ++c) ud[c] = dvar(u[c], c);
        for (int m = 0; m < 15; ++m) qd[m] = dvar(q[m], 5 + m);
        fluxes(ud, qd, nuv, &P, Fc, Fv);

        for (int i = 0; i < Np; ++i) {
            /* gradient equations: rows (3c+j, i) */
            for (int c = 0; c < 5; ++c)
                for (int j = 0; j < 3; ++j) {
                    int row = (3 * c + j) * Np + i;
                    EL(row, colR) += W * (q[3 * c + j] * phi[i] + u[c] * dphi[3 * i + j]);
                    for (int k = 0; k < Np; ++k) {
                        EL(row, (3 * c + j) * Np + k) += W * phi[i] * phi[k];
                        EL(row, (15 + c) * Np + k) += W * dphi[3 * i + j] * phi[k];
                    }
                }
            /* conservation equations: rows (15+c, i) */
            for (int c = 0; c < 5; ++c) {
                int row = (15 + c) * Np + i;
                double res = P.alpha * W * (u[c] - un[c]) * phi[i];
                for (int j = 0; j < 3; ++j)
                    res -= P.dt * W * (Fc[c][j].v - Fv[c][j].v) * dphi[3 * i + j];
                EL(row, colR) += res;
                for (int s = 0; s < 20; ++s) {
                    /* derivative w.r.t. the point value of unknown field s */
                    int slot = (s < 15) ? 5 + s : s - 15;
                    double coef = 0.0;
                    for (int j = 0; j < 3; ++j)
                        coef -= P.dt * W * (Fc[c][j].d[slot] - Fv[c][j].d[slot]) * dphi[3 * i + j];
                    if (s == 15 + c) coef += P.alpha * W * phi[i];
                    if (coef == 0.0) continue;
                    for (int k = 0; k < Np; ++k) EL(row, s * Np + k) += coef * phi[k];
                }
            }
        }
    }

    /* ---------------- face terms ---------------- */
    for (int lf = 0; lf < 6; ++lf) {
        const int d = lf / 2;
        const double sgn = (lf % 2) ? 1.0 : -1.0;
        const int t0 = (d == 0) ? 1 : 0, t1 = (d == 2) ? 1 : 2;
        const int pF = pf[lf], nF = pF + 1, Nfp = nF * nF, nqf = pF + 2;
        double rf[8], xf[8], wf[8];
        hdgref_gll(pF, rf);
        hdgref_gauss(nqf, xf, wf);
        for (int s1 = 0; s1 < nqf; ++s1)
        for (int s0 = 0; s0 < nqf; ++s0) {
            double xi[3];
            xi[d] = sgn;
            xi[t0] = xf[s0];
            xi[t1] = xf[s1];
            double ws = wf[s0] * wf[s1];
            double J[3][3], xx[3], N[3];
            geom_jac(g, Xg, xi, J, xx);
            face_normal(J, d, sgn, N);
            double area = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
            double l[3][8];
            for (int dd = 0; dd < 3; ++dd) lagrange(p, r, xi[dd], l[dd], NULL);
            for (int i2 = 0; i2 < np1; ++i2)
            for (int i1 = 0; i1 < np1; ++i1)
            for (int i0 = 0; i0 < np1; ++i0)
                phi[i0 + np1 * (i1 + np1 * i2)] = l[0][i0] * l[1][i1] * l[2][i2];
            double mu0[8], mu1[8], mu[64];
            lagrange(pF, rf, xf[s0], mu0, NULL);
            lagrange(pF, rf, xf[s1], mu1, NULL);
            for (int a1 = 0; a1 < nF; ++a1)
                for (int a0 = 0; a0 < nF; ++a0) mu[a0 + nF * a1] = mu0[a0] * mu1[a1];
            double u[5] = {0}, q[15] = {0}, uh[5] = {0}, ub[5] = {0}, nuv = 0.0;
            for (int i = 0; i < Np; ++i) {
                for (int c = 0; c < 5; ++c) u[c] += phi[i] * U[c * Np + i];
                for (int m = 0; m < 15; ++m) q[m] += phi[i] * Q[m * Np + i];
                nuv += phi[i] * nu[i];
            }
            for (int c = 0; c < 5; ++c)
                for (int a = 0; a < Nfp; ++a) {
                    uh[c] += mu[a] * Uh[toff[lf] + c * Nfp + a];
                    if (bc[lf] == 1 || bc[lf] == 3) ub[c] += mu[a] * Ub[toff[lf] + c * Nfp + a];
                }
            dual uhd[5], qd[15], Fc[5][3], Fv[5][3], fh[5];
            for (int c = 0; c < 5; ++c) uhd[c] = dvar(uh[c], 20 + c);
            for (int m = 0; m < 15; ++m) qd[m] = dvar(q[m], 5 + m);
            fluxes(uhd, qd, nuv, &P, Fc, Fv);
            for (int c = 0; c < 5; ++c) {
                /* f^ dS = (F^c(uh) - F^v(uh, q)) . N + tau |N| (u - uh) */
                dual fc = dscale(dsub(dvar(u[c], c), uhd[c]), P.tau * area);
                for (int j = 0; j < 3; ++j) fc = dadd(fc, dscale(dsub(Fc[c][j], Fv[c][j]), N[j]));
                fh[c] = fc;
            }
            /* boundary residual b^ of eq. hdg-trace on a boundary face (times |N|):
             *  1 prescribed state:       uh - ub
             *  2 extrapolated state:     uh - u
             *  3 no-slip isothermal wall: (rho^ - rho, m^, rho^E^ - rho^ e_w), e_w the
             *    internal energy of the prescribed state ub
             *  4 no-slip adiabatic wall: (rho^ - rho, m^, f^_energy / |N|)
             *  5 symmetry: (rho^ - rho, m^ - (I - n n^T) m, rho^E^ - rhoE) */
            dual bh[5];
            if (bc[lf]) {
                dual ud[5];
                for (int c = 0; c < 5; ++c) ud[c] = dvar(u[c], c);
                double nn[3] = { N[0] / area, N[1] / area, N[2] / area };
                switch (bc[lf]) {
                case 1:
                    for (int c = 0; c < 5; ++c) bh[c] = dscale(dsub(uhd[c], dconst(ub[c])), area);
                    break;
                case 2:
                    for (int c = 0; c < 5; ++c) bh[c] = dscale(dsub(uhd[c], ud[c]), area);
                    break;
                case 3: case 4: {
                    bh[0] = dscale(dsub(uhd[0], ud[0]), area);
                    for (int i = 1; i < 4; ++i) bh[i] = dscale(uhd[i], area);
                    if (bc[lf] == 3) {
                        double ew = ub[4] / ub[0] - 0.5 * (ub[1] * ub[1] + ub[2] * ub[2] + ub[3] * ub[3]) / (ub[0] * ub[0]);
                        bh[4] = dscale(dsub(uhd[4], dscale(uhd[0], ew)), area);
                    } else {
                        bh[4] = fh[4];
                    }
                    break;
                }
                case 5: {
                    bh[0] = dscale(dsub(uhd[0], ud[0]), area);
                    for (int i = 0; i < 3; ++i) {
                        dual t = uhd[1 + i];
                        for (int j = 0; j < 3; ++j) {
                            double pij = (i == j ? 1.0 : 0.0) - nn[i] * nn[j];
                            t = dsub(t, dscale(ud[1 + j], pij));
                        }
                        bh[1 + i] = dscale(t, area);
                    }
                    bh[4] = dscale(dsub(uhd[4], ud[4]), area);
                    break;
                }
                default:
                    return -1;
                }
            }
            for (int i = 0; i < Np; ++i) {
                if (phi[i] == 0.0) continue;
                /* gradient equations: - < uh, phi_i n_j > */
                for (int c = 0; c < 5; ++c)
                    for (int j = 0; j < 3; ++j) {
                        int row = (3 * c + j) * Np + i;
                        EL(row, colR) -= ws * uh[c] * N[j] * phi[i];
                        for (int a = 0; a < Nfp; ++a)
                            EL(row, n + toff[lf] + c * Nfp + a) -= ws * N[j] * phi[i] * mu[a];
                    }
                /* conservation equations: + dt < f^, phi_i > */
                for (int c = 0; c < 5; ++c) {
                    int row = (15 + c) * Np + i;
                    EL(row, colR) += P.dt * ws * fh[c].v * phi[i];
                    for (int s = 0; s < 20; ++s) {
                        int slot = (s < 15) ? 5 + s : s - 15;
                        double coef = P.dt * ws * fh[c].d[slot] * phi[i];
                        if (coef == 0.0) continue;
                        for (int k = 0; k < Np; ++k) EL(row, s * Np + k) += coef * phi[k];
                    }
                    for (int c2 = 0; c2 < 5; ++c2) {
                        double coef = P.dt * ws * fh[c].d[20 + c2] * phi[i];
                        for (int a = 0; a < Nfp; ++a)
                            EL(row, n + toff[lf] + c2 * Nfp + a) += coef * mu[a];
                    }
                }
            }
            /* trace equations of this element's side of the face */
            for (int c = 0; c < 5; ++c)
                for (int a = 0; a < Nfp; ++a) {
                    int row = n + toff[lf] + c * Nfp + a;
                    /* interior face: < f^, mu >; boundary face: < b^, mu > */
                    const dual *r = bc[lf] ? bh : fh;
                    EL(row, colR) += ws * r[c].v * mu[a];
                    for (int s = 0; s < 20; ++s) {
                        int slot = (s < 15) ? 5 + s : s - 15;
                        double coef = ws * r[c].d[slot] * mu[a];
                        if (coef == 0.0) continue;
                        for (int k = 0; k < Np; ++k) EL(row, s * Np + k) += coef * phi[k];
                    }
                    for (int c2 = 0; c2 < 5; ++c2)
                        for (int b = 0; b < Nfp; ++b)
                            EL(row, n + toff[lf] + c2 * Nfp + b) += ws * r[c].d[20 + c2] * mu[a] * mu[b];
                }
        }
    }
    free(phi);
    free(dphi);
#undef EL
    return 0;
}

/* Volume quadrature data for pins: |K| and the element mass matrix row sums. */
double hdgref_element_volume(int p, int g, const double *Xg)
{
    double xg[8], wg[8];
    hdgref_gauss(p + 2, xg, wg);
    double vol = 0.0;
    for (int g2 = 0; g2 < p + 2; ++g2)
        for (int g1 = 0; g1 < p + 2; ++g1)
            for (int g0 = 0; g0 < p + 2; ++g0) {
                double xi[3] = { xg[g0], xg[g1], xg[g2] }, J[3][3], G[3][3], xx[3];
                geom_jac(g, Xg, xi, J, xx);
                vol += wg[g0] * wg[g1] * wg[g2] * inv3(J, G);
            }
    return vol;
}

/* ------------------------------------------------------------------ */
/* Static condensation (eqs. local-elimination, schur-trace)           */
/* ------------------------------------------------------------------ */
/* In-place LU with partial pivoting of the n x n column-major matrix a (lda).
 * Returns 0, or k+1 if the k-th pivot is exactly zero. */
static int lu_factor(int n, double *a, int lda, int *piv)
{
    int info = 0;
    for (int k = 0; k < n; ++k) {
        int pr = k;
        double best = fabs(a[k + (size_t)k * lda]);
        for (int i = k + 1; i < n; ++i) {
            double v = fabs(a[i + (size_t)k * lda]);
            if (v > best) { best = v; pr = i; }
        }
        piv[k] = pr;
        if (best == 0.0) { if (!info) info = k + 1; continue; }
        if (pr != k)
            for (int j = 0; j < n; ++j) {
                double t = a[k + (size_t)j * lda];
                a[k + (size_t)j * lda] = a[pr + (size_t)j * lda];
                a[pr + (size_t)j * lda] = t;
            }
        double inv = 1.0 / a[k + (size_t)k * lda];
        for (int i = k + 1; i < n; ++i) a[i + (size_t)k * lda] *= inv;
        for (int j = k + 1; j < n; ++j) {
            double ukj = a[k + (size_t)j * lda];
            if (ukj == 0.0) continue;
            double *cj = a + (size_t)j * lda, *ck = a + (size_t)k * lda;
            for (int i = k + 1; i < n; ++i) cj[i] -= ck[i] * ukj;
        }
    }
    return info;
}

/* Solve (LU) x = P b for nrhs columns of b (ldb), in place. */
static void lu_solve(int n, const double *a, int lda, const int *piv, double *b, int ldb, int nrhs)
{
    for (int r = 0; r < nrhs; ++r) {
        double *x = b + (size_t)r * ldb;
        for (int k = 0; k < n; ++k)
            if (piv[k] != k) { double t = x[k]; x[k] = x[piv[k]]; x[piv[k]] = t; }
        for (int j = 0; j < n; ++j) {
            double xj = x[j];
            if (xj == 0.0) continue;
            const double *cj = a + (size_t)j * lda;
            for (int i = j + 1; i < n; ++i) x[i] -= cj[i] * xj;
        }
        for (int j = n - 1; j >= 0; --j) {
            x[j] /= a[j + (size_t)j * lda];
            double xj = x[j];
            const double *cj = a + (size_t)j * lda;
            for (int i = 0; i < j; ++i) x[i] -= cj[i] * xj;
        }
    }
}

/*
 * From the element system E (layout above): X = A^{-1} [B | R_qu] (n x (f+1),
 * column-major), S^K = D - C X_B (f x f, column-major), g^K = -R_uh + C x_r.
 * Returns the LU info (0 on success).
 */
int hdgref_condense(int n, int f, const double *E, double *SK, double *gK, double *X)
{
    const int ld = n + f;
    double *A = malloc(sizeof(double) * (size_t)n * n);
    int *piv = malloc(sizeof(int) * n);
    for (int j = 0; j < n; ++j)
        memcpy(A + (size_t)j * n, E + (size_t)j * ld, sizeof(double) * n);
    int info = lu_factor(n, A, n, piv);
    for (int j = 0; j <= f; ++j)
        memcpy(X + (size_t)j * n, E + (size_t)(n + j) * ld, sizeof(double) * n);
    if (!info) lu_solve(n, A, n, piv, X, n, f + 1);
    /* S = D - C X_B ; g = -R_uh + C x_r */
    for (int j = 0; j <= f; ++j) {
        double *out = (j < f) ? SK + (size_t)j * f : gK;
        const double *src = E + n + (size_t)(n + j) * ld;  /* D column j or R_uh */
        for (int i = 0; i < f; ++i) out[i] = (j < f) ? src[i] : -src[i];
        const double *xj = X + (size_t)j * n;
        double sgn = (j < f) ? -1.0 : 1.0;
        for (int k = 0; k < n; ++k) {
            double xk = xj[k];
            if (xk == 0.0) continue;
            const double *ck = E + n + (size_t)k * ld;  /* C column k */
            for (int i = 0; i < f; ++i) out[i] += sgn * ck[i] * xk;
        }
    }
    free(A);
    free(piv);
    return info;
}

/* Factor once, solve many times (the additive-Schwarz blocks inside GMRES):
 * the same LU with partial pivoting as above, exposed in two calls. */
int hdgref_lu_factor(int n, double *a, int *piv) { return lu_factor(n, a, n, piv); }
void hdgref_lu_solve(int n, const double *a, const int *piv, double *b, int nrhs)
{
    lu_solve(n, a, n, piv, b, n, nrhs);
}

/* Dense LU solve of a general system (used for the additive-Schwarz blocks and
 * the brute-force check): solves a x = b in place for nrhs columns. */
int hdgref_dense_solve(int n, double *a, double *b, int nrhs)
{
    int *piv = malloc(sizeof(int) * n);
    int info = lu_factor(n, a, n, piv);
    if (!info) lu_solve(n, a, n, piv, b, n, nrhs);
    free(piv);
    return info;
}
