// Element residuals and Jacobian blocks of the HDG discretisation.
//
// Two stages (the quadrature-point kernels feed the assembly kernel through a
// workspace, as in the paper's split of pointwise kernels and assembly
// kernels that look like batched linear algebra):
//   k_qp_volume / k_qp_face : interpolate (u, u^n, q, nu) to the Gauss points,
//       evaluate the fluxes of eqs. convective-flux, viscous-flux, stress-heat,
//       av-total and the numerical flux of eq. num-flux-hdg, and their exact
//       Jacobians (derived by hand below), already multiplied by quadrature
//       weights, the geometric factors and dt / alpha;
//   k_assemble_field_rows / k_assemble_trace_rows : contract the point
//       coefficients with the basis (phi_i, reference derivatives of phi_i,
//       phi_k, trace basis mu_a) into the rows of the element system
//       E^K = [[A B R_qu],[C D R_uh]], by sum factorisation over the tensor
//       Gauss points.  Their bulk stores are nontemporal: a chunk's systems
//       (21.7 GB for 256 elements at p = 4) are far larger than any cache, so
//       keeping the written lines only evicts other data.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "hdg_internal.h"

namespace hdg {
namespace {

typedef double v2d __attribute__((ext_vector_type(2)));

// ------------------------------------------------------------------ physics
// Intermediates at one point for state w and conservative gradient q.
struct PState {
    double rho, v[3], E, mus, kap, dmus[5];
    double dv[3][3], dE[3], de[3], S[3][3];
    double vv;  // |v|^2
};

__device__ inline void pstate(const double *w, const double *q, const Phys &P, PState &s) {
    const double rho = w[0], ir = 1.0 / rho;
    s.rho = rho;
    for (int i = 0; i < 3; ++i) s.v[i] = w[1 + i] * ir;
    s.E = w[4] * ir;
    s.vv = s.v[0] * s.v[0] + s.v[1] * s.v[1] + s.v[2] * s.v[2];
    const double e = s.E - 0.5 * s.vv;
    const double cT = P.gamma * (P.gamma - 1.0) * P.mach * P.mach;
    double mu = 1.0, dmu = 0.0;
    if (P.visc_law == 1) {
        const double T = cT * e, sq = sqrt(T), den = 1.0 / (T + 0.40417);
        mu = 1.4042 * T * sq * den;
        // d/dT [c1 T^{3/2} / (T + c2)] = c1 sqrt(T) (T/2 + 3 c2 / 2) / (T + c2)^2
        dmu = 1.4042 * sq * (0.5 * T + 1.5 * 0.40417) * den * den;
    }
    s.mus = mu / P.reynolds;
    s.kap = P.gamma * s.mus / P.prandtl;
    // de/dw = ((|v|^2 - E)/rho, -v/rho, 1/rho)
    const double dedw[5] = {(s.vv - s.E) * ir, -s.v[0] * ir, -s.v[1] * ir, -s.v[2] * ir, ir};
    for (int c = 0; c < 5; ++c) s.dmus[c] = dmu * cT * dedw[c] / P.reynolds;
    for (int j = 0; j < 3; ++j) {
        for (int i = 0; i < 3; ++i) s.dv[i][j] = (q[3 * (1 + i) + j] - s.v[i] * q[j]) * ir;
        s.dE[j] = (q[12 + j] - s.E * q[j]) * ir;
        s.de[j] = s.dE[j] - (s.v[0] * s.dv[0][j] + s.v[1] * s.dv[1][j] + s.v[2] * s.dv[2][j]);
    }
    const double div = s.dv[0][0] + s.dv[1][1] + s.dv[2][2];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) s.S[i][j] = s.dv[i][j] + s.dv[j][i] - (i == j ? (2.0 / 3.0) * div : 0.0);
}

// F = F^c(w) - F^v(w, q) - nu q   (total flux entering the residuals)
__device__ inline void total_flux(const double *w, const double *q, double nu, const Phys &P,
                                  const PState &s, double F[5][3]) {
    const double p = (P.gamma - 1.0) * (w[4] - 0.5 * s.rho * s.vv);
    for (int j = 0; j < 3; ++j) {
        F[0][j] = w[1 + j];
        double tv = 0.0;
        for (int i = 0; i < 3; ++i) {
            const double tau = s.mus * s.S[i][j];
            F[1 + i][j] = w[1 + i] * s.v[j] + (i == j ? p : 0.0) - tau;
            tv += s.v[i] * tau;
        }
        F[4][j] = (w[4] + p) * s.v[j] - tv - s.kap * s.de[j];
        for (int c = 0; c < 5; ++c) F[c][j] -= nu * q[3 * c + j];
    }
}

// dF/dw_cp (q fixed) of F = F^c - F^v; nu q does not depend on w.
__device__ inline void dflux_dw(const double *w, const double *q, const Phys &P, const PState &s,
                                int cp, double dF[5][3]) {
    const double ir = 1.0 / s.rho, gm1 = P.gamma - 1.0;
    const double p = gm1 * (w[4] - 0.5 * s.rho * s.vv);
    double dp, dvel[3];
    if (cp == 0) {
        dp = gm1 * 0.5 * s.vv;
        for (int i = 0; i < 3; ++i) dvel[i] = -s.v[i] * ir;
    } else if (cp < 4) {
        dp = -gm1 * s.v[cp - 1];
        for (int i = 0; i < 3; ++i) dvel[i] = (i == cp - 1) ? ir : 0.0;
    } else {
        dp = gm1;
        for (int i = 0; i < 3; ++i) dvel[i] = 0.0;
    }
    // derivatives of the primitive gradients
    double ddv[3][3], ddE[3], dde[3];
    for (int j = 0; j < 3; ++j) {
        const double q0 = q[j];
        for (int i = 0; i < 3; ++i) {
            if (cp == 0) ddv[i][j] = (s.v[i] * q0 * ir - s.dv[i][j]) * ir;
            else if (cp == 1 + i) ddv[i][j] = -q0 * ir * ir;
            else ddv[i][j] = 0.0;
        }
        if (cp == 0) ddE[j] = (s.E * q0 * ir - s.dE[j]) * ir;
        else if (cp == 4) ddE[j] = -q0 * ir * ir;
        else ddE[j] = 0.0;
        dde[j] = ddE[j];
        for (int i = 0; i < 3; ++i) dde[j] -= dvel[i] * s.dv[i][j] + s.v[i] * ddv[i][j];
    }
    const double ddiv = ddv[0][0] + ddv[1][1] + ddv[2][2];
    const double dmus = s.dmus[cp], dkap = P.gamma * dmus / P.prandtl;
    for (int j = 0; j < 3; ++j) {
        // convective part
        dF[0][j] = (cp == 1 + j) ? 1.0 : 0.0;
        for (int i = 0; i < 3; ++i)
            dF[1 + i][j] = ((cp == 1 + i) ? s.v[j] : 0.0) + s.rho * s.v[i] * dvel[j] + (i == j ? dp : 0.0);
        dF[4][j] = ((cp == 4 ? 1.0 : 0.0) + dp) * s.v[j] + (w[4] + p) * dvel[j];
        // viscous part
        double dvt = 0.0;
        for (int i = 0; i < 3; ++i) {
            const double dS = ddv[i][j] + ddv[j][i] - (i == j ? (2.0 / 3.0) * ddiv : 0.0);
            const double dtau = dmus * s.S[i][j] + s.mus * dS;
            dF[1 + i][j] -= dtau;
            dvt += dvel[i] * s.mus * s.S[i][j] + s.v[i] * dtau;
        }
        dF[4][j] -= dvt + dkap * s.de[j] + s.kap * dde[j];
    }
}

// dF^v/dq_{cpp,l} including nu q (F^v is linear in q).
__device__ inline void dfv_dq(const PState &s, double nu, int cpp, int l, double dF[5][3]) {
    const double ir = 1.0 / s.rho;
    double b[3];
    for (int i = 0; i < 3; ++i) b[i] = (((cpp == 1 + i) ? 1.0 : 0.0) - (cpp == 0 ? s.v[i] : 0.0)) * ir;
    double a = 0.0;
    if (cpp == 4) a = ir;
    else if (cpp == 0) a = (s.vv - s.E) * ir;
    else a = -s.v[cpp - 1] * ir;
    const double vb = s.v[0] * b[0] + s.v[1] * b[1] + s.v[2] * b[2];
    for (int j = 0; j < 3; ++j) {
        const double djl = (j == l) ? 1.0 : 0.0;
        dF[0][j] = (cpp == 0) ? nu * djl : 0.0;
        for (int i = 0; i < 3; ++i)
            dF[1 + i][j] = s.mus * (djl * b[i] + (i == l ? b[j] : 0.0) - (i == j ? (2.0 / 3.0) * b[l] : 0.0)) +
                           ((cpp == 1 + i) ? nu * djl : 0.0);
        dF[4][j] = s.mus * (djl * vb + s.v[l] * b[j] - (2.0 / 3.0) * s.v[j] * b[l]) + s.kap * djl * a +
                   ((cpp == 4) ? nu * djl : 0.0);
    }
}

__device__ inline int64_t qp_face_base(const DevMesh &dm, int e, int lf, int Nq) {
    int64_t off = dm.qp_off[e] + (int64_t)(kVJac + kVRes) * Nq;
    for (int l = 0; l < lf; ++l) {
        const int pf = dm.face_p[dm.elem_face[6 * e + l]];
        off += (int64_t)kFPer * (pf + 2) * (pf + 2);
    }
    return off;
}

// ------------------------------------------------------- point kernel: volume
__global__ void __launch_bounds__(256) k_qp_volume(DevMesh dm, Phys P, int e0, const double *__restrict__ Qg,
                                                   const double *__restrict__ Ug, const double *__restrict__ Ung,
                                                   const double *__restrict__ nug, double *__restrict__ qp) {
    const int e = e0 + blockIdx.x;
    const int p = dm.elem_p[e], p1 = p + 1, Np = p1 * p1 * p1, nq = p + 2, Nq = nq * nq * nq;
    __shared__ double sU[5 * 125], sUn[5 * 125], sQ[15 * 125], sNu[125], sL[5 * 6];
    const int64_t no = dm.node_off[e];
    for (int t = threadIdx.x; t < 5 * Np; t += blockDim.x) {
        sU[t] = Ug[5 * no + t];
        sUn[t] = Ung[5 * no + t];
    }
    for (int t = threadIdx.x; t < 15 * Np; t += blockDim.x) sQ[t] = Qg[15 * no + t];
    for (int t = threadIdx.x; t < Np; t += blockDim.x) sNu[t] = nug[no + t];
    for (int t = threadIdx.x; t < p1 * nq; t += blockDim.x) sL[t] = dm.tbl[tbl_L(p, p, t / nq, t % nq)];
    __syncthreads();
    const double *vg = dm.vgeo + dm.vgeo_off[e];
    double *out = qp + (dm.qp_off[e] - dm.qp_off[e0]);
    for (int g = threadIdx.x; g < Nq; g += blockDim.x) {
        const int g0 = g % nq, g1 = (g / nq) % nq, g2 = g / (nq * nq);
        double u[5] = {0, 0, 0, 0, 0}, un[5] = {0, 0, 0, 0, 0}, q[15], nu = 0.0;
        for (int m = 0; m < 15; ++m) q[m] = 0.0;
        for (int i2 = 0; i2 < p1; ++i2)
            for (int i1 = 0; i1 < p1; ++i1) {
                const double l12 = sL[i1 * nq + g1] * sL[i2 * nq + g2];
                for (int i0 = 0; i0 < p1; ++i0) {
                    const double ph = sL[i0 * nq + g0] * l12;
                    const int i = i0 + p1 * (i1 + p1 * i2);
                    for (int c = 0; c < 5; ++c) {
                        u[c] += ph * sU[c * Np + i];
                        un[c] += ph * sUn[c * Np + i];
                    }
                    for (int m = 0; m < 15; ++m) q[m] += ph * sQ[m * Np + i];
                    nu += ph * sNu[i];
                }
            }
        const double W = vg[g];
        double G[3][3];
        for (int d = 0; d < 3; ++d)
            for (int j = 0; j < 3; ++j) G[d][j] = vg[(1 + 3 * d + j) * Nq + g];
        PState s;
        pstate(u, q, P, s);
        double F[5][3];
        total_flux(u, q, nu, P, s, F);
        double *vres = out + (int64_t)kVJac * Nq;
        // residual coefficients: gradient rows
        for (int c = 0; c < 5; ++c)
            for (int j = 0; j < 3; ++j) {
                const int r = 3 * c + j;
                vres[(4 * r + 0) * Nq + g] = W * q[r];
                for (int d = 0; d < 3; ++d) vres[(4 * r + 1 + d) * Nq + g] = W * u[c] * G[d][j];
            }
        // residual coefficients: conservation rows
        for (int c = 0; c < 5; ++c) {
            const int r = 15 + c;
            vres[(4 * r + 0) * Nq + g] = P.alpha * W * (u[c] - un[c]);
            for (int d = 0; d < 3; ++d)
                vres[(4 * r + 1 + d) * Nq + g] = -P.dt * W * (G[d][0] * F[c][0] + G[d][1] * F[c][1] + G[d][2] * F[c][2]);
        }
        // Jacobian coefficients of the conservation rows
        for (int cp = 0; cp < 5; ++cp) {
            double dF[5][3];
            dflux_dw(u, q, P, s, cp, dF);
            for (int c = 0; c < 5; ++c) {
                const int sidx = 15 + cp;
                double *o = out + (int64_t)(4 * (20 * c + sidx)) * Nq + g;
                o[0] = (c == cp) ? P.alpha * W : 0.0;
                for (int d = 0; d < 3; ++d)
                    o[(1 + d) * Nq] = -P.dt * W * (G[d][0] * dF[c][0] + G[d][1] * dF[c][1] + G[d][2] * dF[c][2]);
            }
        }
        for (int m = 0; m < 15; ++m) {
            double dF[5][3];
            dfv_dq(s, nu, m / 3, m % 3, dF);
            for (int c = 0; c < 5; ++c) {
                double *o = out + (int64_t)(4 * (20 * c + m)) * Nq + g;
                o[0] = 0.0;
                for (int d = 0; d < 3; ++d)
                    o[(1 + d) * Nq] = P.dt * W * (G[d][0] * dF[c][0] + G[d][1] * dF[c][1] + G[d][2] * dF[c][2]);
            }
        }
    }
}

// --------------------------------------------------------- point kernel: face
__global__ void __launch_bounds__(64) k_qp_face(DevMesh dm, Phys P, int e0, const double *__restrict__ Qg,
                                                const double *__restrict__ Ug, const double *__restrict__ Uhg,
                                                const double *__restrict__ nug, const double *__restrict__ Ubg,
                                                double *__restrict__ qp) {
    const int lf = blockIdx.x, e = e0 + blockIdx.y;
    const int p = dm.elem_p[e], p1 = p + 1, Np = p1 * p1 * p1, nq = p + 2, Nq = nq * nq * nq;
    const int F = dm.elem_face[6 * e + lf], pf = dm.face_p[F], pf1 = pf + 1, nqf1 = pf + 2, Nqf = nqf1 * nqf1;
    const int Nfp = pf1 * pf1, bc = dm.face_bc[F];
    const int d = lf / 2, side = lf & 1, t0 = (d == 0) ? 1 : 0, t1 = (d == 2) ? 1 : 2;
    const int64_t no = dm.node_off[e];
    const double *fg = dm.fgeo + dm.fgeo_off[6 * e + lf];
    double *out = qp + (qp_face_base(dm, e, lf, Nq) - dm.qp_off[e0]);
    const double *uh_g = Uhg + dm.face_off[F];
    const bool has_ub = (bc == 1 || bc == 3);  // boundary types that read prescribed data
    const double *ub_g = has_ub ? Ubg + dm.face_off[F] : nullptr;
    for (int s = threadIdx.x; s < Nqf; s += blockDim.x) {
        const int s0 = s % nqf1, s1 = s / nqf1;
        double u[5] = {0, 0, 0, 0, 0}, q[15], nu = 0.0, uh[5] = {0, 0, 0, 0, 0}, ub[5] = {0, 0, 0, 0, 0};
        for (int m = 0; m < 15; ++m) q[m] = 0.0;
        // element fields: only the nodes on this face are nonzero there
        for (int a1 = 0; a1 < p1; ++a1)
            for (int a0 = 0; a0 < p1; ++a0) {
                const double ph = dm.tbl[tbl_L(p, pf, a0, s0)] * dm.tbl[tbl_L(p, pf, a1, s1)];
                int idx[3];
                idx[d] = side ? p : 0;
                idx[t0] = a0;
                idx[t1] = a1;
                const int i = idx[0] + p1 * (idx[1] + p1 * idx[2]);
                for (int c = 0; c < 5; ++c) u[c] += ph * Ug[5 * no + c * Np + i];
                for (int m = 0; m < 15; ++m) q[m] += ph * Qg[15 * no + m * Np + i];
                nu += ph * nug[no + i];
            }
        for (int b1 = 0; b1 < pf1; ++b1)
            for (int b0 = 0; b0 < pf1; ++b0) {
                const double mu = dm.tbl[tbl_L(pf, pf, b0, s0)] * dm.tbl[tbl_L(pf, pf, b1, s1)];
                const int b = b0 + pf1 * b1;
                for (int c = 0; c < 5; ++c) {
                    uh[c] += mu * uh_g[c * Nfp + b];
                    if (has_ub) ub[c] += mu * ub_g[c * Nfp + b];
                }
            }
        const double wN[3] = {fg[s], fg[Nqf + s], fg[2 * Nqf + s]}, wA = fg[3 * Nqf + s];
        PState st;
        pstate(uh, q, P, st);
        double Fl[5][3];
        total_flux(uh, q, nu, P, st, Fl);
        for (int c = 0; c < 5; ++c) {
            out[(125 + c) * Nqf + s] = Fl[c][0] * wN[0] + Fl[c][1] * wN[1] + Fl[c][2] * wN[2] + P.tau * wA * (u[c] - uh[c]);
            out[(130 + c) * Nqf + s] = 0.0;
            out[(135 + c) * Nqf + s] = uh[c];
        }
        // d fh / d u (element trace): tau |N| I
        for (int c = 0; c < 5; ++c)
            for (int cp = 0; cp < 5; ++cp) out[(25 * c + cp) * Nqf + s] = (c == cp) ? P.tau * wA : 0.0;
        // d fh / d q
        for (int m = 0; m < 15; ++m) {
            double dF[5][3];
            dfv_dq(st, nu, m / 3, m % 3, dF);
            for (int c = 0; c < 5; ++c)
                out[(25 * c + 5 + m) * Nqf + s] = -(dF[c][0] * wN[0] + dF[c][1] * wN[1] + dF[c][2] * wN[2]);
        }
        // d fh / d uh
        for (int cp = 0; cp < 5; ++cp) {
            double dF[5][3];
            dflux_dw(uh, q, P, st, cp, dF);
            for (int c = 0; c < 5; ++c)
                out[(25 * c + 20 + cp) * Nqf + s] =
                    dF[c][0] * wN[0] + dF[c][1] * wN[1] + dF[c][2] * wN[2] - ((c == cp) ? P.tau * wA : 0.0);
        }
        if (bc) {
            // boundary residual b^ of eq. hdg-trace (weighted by w |N|) into slots 130+c, its
            // derivatives d b^_c / d(u 0..4, q 5..19, uh 20..24) into 140 + 25 c + slot:
            //  1 prescribed state uh - ub; 2 extrapolated state uh - u;
            //  3 no-slip isothermal wall (rho^ - rho, m^, rho^E^ - rho^ e_w), e_w the internal
            //    energy of the prescribed state; 4 no-slip adiabatic wall (rho^ - rho, m^, the
            //    energy component of the numerical flux); 5 symmetry (rho^ - rho,
            //    m^ - (I - n n^T) m, rho^E^ - rhoE)
            double *bj = out + (int64_t)140 * Nqf + s;
            for (int k = 0; k < 125; ++k) bj[(int64_t)k * Nqf] = 0.0;
            auto J = [&](int c, int slot) -> double & { return bj[(int64_t)(25 * c + slot) * Nqf]; };
            double br[5];
            if (bc == 1 || bc == 2) {
                for (int c = 0; c < 5; ++c) {
                    br[c] = wA * (uh[c] - (bc == 1 ? ub[c] : u[c]));
                    J(c, 20 + c) = wA;
                    if (bc == 2) J(c, c) = -wA;
                }
            } else if (bc == 3 || bc == 4) {
                br[0] = wA * (uh[0] - u[0]);
                J(0, 20) = wA;
                J(0, 0) = -wA;
                for (int i = 1; i < 4; ++i) {
                    br[i] = wA * uh[i];
                    J(i, 20 + i) = wA;
                }
                if (bc == 3) {
                    const double ew = ub[4] / ub[0] - 0.5 * (ub[1] * ub[1] + ub[2] * ub[2] + ub[3] * ub[3]) / (ub[0] * ub[0]);
                    br[4] = wA * (uh[4] - ew * uh[0]);
                    J(4, 24) = wA;
                    J(4, 20) = -wA * ew;
                } else {
                    br[4] = out[(125 + 4) * Nqf + s];
                    for (int k = 0; k < 25; ++k) J(4, k) = out[(25 * 4 + k) * Nqf + s];
                }
            } else {
                const double nn[3] = {wN[0] / wA, wN[1] / wA, wN[2] / wA};
                br[0] = wA * (uh[0] - u[0]);
                J(0, 20) = wA;
                J(0, 0) = -wA;
                for (int i = 0; i < 3; ++i) {
                    double t = uh[1 + i];
                    for (int j = 0; j < 3; ++j) {
                        const double pij = (i == j ? 1.0 : 0.0) - nn[i] * nn[j];
                        t -= pij * u[1 + j];
                        J(1 + i, 1 + j) = -wA * pij;
                    }
                    br[1 + i] = wA * t;
                    J(1 + i, 21 + i) = wA;
                }
                br[4] = wA * (uh[4] - u[4]);
                J(4, 24) = wA;
                J(4, 4) = -wA;
            }
            for (int c = 0; c < 5; ++c) out[(130 + c) * Nqf + s] = br[c];
        }
    }
}

// --------------------------------------------------------- assembly kernel
// Face of an element: is volume node i on local face lf, and its face indices.
__device__ inline bool on_face(int i, int p1, int lf, int &a0, int &a1) {
    const int d = lf / 2, side = lf & 1;
    int idx[3] = {i % p1, (i / p1) % p1, i / (p1 * p1)};
    if (idx[d] != (side ? p1 - 1 : 0)) return false;
    const int t0 = (d == 0) ? 1 : 0, t1 = (d == 2) ? 1 : 2;
    a0 = idx[t0];
    a1 = idx[t1];
    return true;
}



// Face tables of the element-row kernels: the element's 1-D basis and each
// face's trace basis at the face's Gauss points, face quadrature bases in the
// point workspace.
__device__ inline void load_face_tables(const DevMesh &dm, int e, int p, int Nq, double (*sLf)[30],
                                        double (*sMf)[30], int *sPf, int *sNqf, int64_t *sFbase) {
    const int tid = threadIdx.x;
    if (tid < 6) {
        const int pf = dm.face_p[dm.elem_face[6 * e + tid]];
        sPf[tid] = pf;
        sNqf[tid] = (pf + 2) * (pf + 2);
        sFbase[tid] = qp_face_base(dm, e, tid, Nq) - dm.qp_off[e];
    }
    __syncthreads();
    for (int t = tid; t < 6 * 30; t += blockDim.x) {
        const int lf = t / 30, r = t % 30, pf = sPf[lf], nqf1 = pf + 2;
        const int a = r / nqf1, s = r % nqf1;
        sLf[lf][r] = (r < (p + 1) * nqf1) ? dm.tbl[tbl_L(p, pf, a, s)] : 0.0;
        sMf[lf][r] = (r < (pf + 1) * nqf1) ? dm.tbl[tbl_L(pf, pf, a, s)] : 0.0;
    }
}

// Interior rows of one row field r of the element system (the workgroups that
// share it are described below the helpers): the 20 column blocks of A, the
// trace columns B, the residual column and the padding, all written.  Gradient rows r = 3c+j hold the mass
// block (column field r) and K_j = int phi_k d_j phi_i (column field 15+c) and
// zeros elsewhere; conservation rows r = 15+c hold the blocks of the point
// Jacobians plus their face terms.
//
// Every N_p x N_p block sum_g phi_k(g) [c0 phi_i + sum_d c_d dref_d phi_i](g) is
// contracted one direction at a time over the tensor Gauss points (sum
// factorisation), one i1 slice at a time:
//   x:  T0 = sum_g1 (L_i1 c0 + D_i1 c1) L_k1,  T2 = sum_g1 L_i1 c2 L_k1,  T3 = sum_g1 L_i1 c3 L_k1
//   y:  VL = sum_g2 (L_i2 T0 + D_i2 T2) L_k2,   VD = sum_g2 L_i2 T3 L_k2
//   z:  A  = sum_g3 (L_i3 VL + D_i3 VD) L_k3
// (L, D: the 1-D basis and its derivative at the Gauss points).  The face terms
// and the trace columns are 2-D contractions over each face's Gauss points.
constexpr int kP1 = kMaxP + 1, kNQ = kMaxP + 2;

// Instantiated per degree PT (LDS sized for it, loop bounds and index arithmetic
// known at compile time); workgroups of elements of another degree return.
// Row fields 0..14 (q) take one workgroup each; each of the five u row fields,
// whose 20 column-field blocks all carry volume and face terms, is split over
// kUG workgroups by column fields (the first of them also writes the trace
// columns, the residual column and the padding).  The launch has 15 + 5 kUG
// workgroups per element.
constexpr int kUG = 4;
template <int PT>
__global__ void __launch_bounds__(256) k_assemble_field_rows(DevMesh dm, Phys P, int e0, const double *__restrict__ qp,
                                                             double *__restrict__ Ebase) {
    const int bx = blockIdx.x, e = e0 + blockIdx.y;
    const int r = bx < 15 ? bx : 15 + (bx - 15) / kUG;  // row field
    const int ug = bx < 15 ? 0 : (bx - 15) % kUG;        // column-field group of a u row
    if (dm.elem_p[e] != PT) return;
    constexpr int p = PT, p1 = p + 1, Np = p1 * p1 * p1, nq = p + 2, Nq = nq * nq * nq;
    // face-term blocks (6 p1^4) and trace-column blocks (5 p1^2 Nfp, face degree up to kMaxP)
    constexpr int kSF = std::max(6 * p1 * p1 * p1 * p1, 5 * p1 * p1 * kP1 * kP1);
    constexpr int kSG = std::max(6 * p1 * p1 * kNQ, 5 * p1 * kP1 * kNQ);
    const int *toff = dm.toff + 7 * e;
    const int n = 20 * Np, f = toff[6];
    const int64_t ld = e_ld(n, f);
    double *E = Ebase + (dm.E_off[e] - dm.E_off[e0]);
    double *Er = E + (int64_t)r * Np * ld;
    const double *qpe = qp + (dm.qp_off[e] - dm.qp_off[e0]);
    const double *vg = dm.vgeo + dm.vgeo_off[e];
    const int tid = threadIdx.x;
    const bool qrow = r < 15;
    const int c = qrow ? r / 3 : r - 15, jdir = qrow ? r % 3 : 0;

    __shared__ double sL[p1][nq], sD[p1][nq];
    __shared__ double sLf[6][30], sMf[6][30];
    __shared__ int sPf[6], sNqf[6];
    __shared__ int64_t sFbase[6];
    __shared__ double sC[4][Nq];                 // coefficient fields of one block
    __shared__ double sT[3][p1][nq * nq];        // x stage of one i1 slice
    __shared__ double sV[2][p1 * p1 * p1][nq];   // y stage of one i1 slice
    __shared__ double sF[kSF];                   // face terms / trace-column blocks
    __shared__ double sG[kSG];                   // first stage of the 2-D contractions
    constexpr int kNqfFace = kNQ * kNQ;          // Gauss points of a face, at most
    __shared__ double sCf[6][kNqfFace];          // one block's face coefficients
    __shared__ unsigned char sNm[Np];            // faces each node lies on (bit lf)
    __shared__ unsigned char sNa[6][Np];         // its face-local index a0 p1 + a1 there
    for (int t = tid; t < p1 * nq; t += blockDim.x) {
        sL[t / nq][t % nq] = dm.tbl[tbl_L(p, p, t / nq, t % nq)];
        sD[t / nq][t % nq] = dm.tbl[tbl_D(p, t / nq, t % nq)];
    }
    for (int i = tid; i < Np; i += blockDim.x) {
        const int idx[3] = {i % p1, (i / p1) % p1, i / (p1 * p1)};
        unsigned m = 0;
        for (int lf = 0; lf < 6; ++lf) {
            const int d = lf >> 1;
            if (idx[d] == ((lf & 1) ? p : 0)) {
                m |= 1u << lf;
                const int a0 = (d == 0) ? idx[1] : idx[0], a1 = (d == 2) ? idx[1] : idx[2];
                sNa[lf][i] = (unsigned char)(a0 * p1 + a1);
            } else {
                sNa[lf][i] = 0;
            }
        }
        sNm[i] = (unsigned char)m;
    }
    load_face_tables(dm, e, p, Nq, sLf, sMf, sPf, sNqf, sFbase);
    __syncthreads();

    // face-tangential indices (a0, a1) of volume node (i1, i2, i3) on face lf, or false
    auto face_idx = [&](int i1, int i2, int i3, int lf, int &a0, int &a1) {
        const int d = lf >> 1, v = (lf & 1) ? p : 0;
        const int id = (d == 0) ? i1 : ((d == 1) ? i2 : i3);
        if (id != v) return false;
        a0 = (d == 0) ? i2 : i1;
        a1 = (d == 2) ? i2 : i3;
        return true;
    };

    // one sum-factorised block from sC into column field sblk (with the face terms in sF)
    auto volume_block = [&](int sblk, bool faces) {
        for (int i1 = 0; i1 < p1; ++i1) {
            __syncthreads();
            for (int t = tid; t < p1 * nq * nq; t += blockDim.x) {
                const int k1 = t / (nq * nq), g23 = t % (nq * nq);
                double a0 = 0.0, a2 = 0.0, a3 = 0.0;
                for (int g1 = 0; g1 < nq; ++g1) {
                    const int g = g1 + nq * g23;
                    const double lk = sL[k1][g1], li = sL[i1][g1];
                    a0 += (li * sC[0][g] + sD[i1][g1] * sC[1][g]) * lk;
                    a2 += li * sC[2][g] * lk;
                    a3 += li * sC[3][g] * lk;
                }
                sT[0][k1][g23] = a0;
                sT[1][k1][g23] = a2;
                sT[2][k1][g23] = a3;
            }
            __syncthreads();
            for (int t = tid; t < p1 * p1 * p1 * nq; t += blockDim.x) {
                const int g3 = t % nq, q = t / nq;  // q = (i2 p1 + k1) p1 + k2
                const int k2 = q % p1, k1 = (q / p1) % p1, i2 = q / (p1 * p1);
                double vl = 0.0, vd = 0.0;
                for (int g2 = 0; g2 < nq; ++g2) {
                    const int g23 = g2 + nq * g3;
                    const double lk = sL[k2][g2];
                    vl += (sL[i2][g2] * sT[0][k1][g23] + sD[i2][g2] * sT[1][k1][g23]) * lk;
                    vd += sL[i2][g2] * sT[2][k1][g23] * lk;
                }
                sV[0][q][g3] = vl;
                sV[1][q][g3] = vd;
            }
            __syncthreads();
            if constexpr (p1 * p1 * p1 * p1 <= 256) {
                // one pass of the workgroup: a thread takes the p1 outputs k = k12 + p1^2 k3
                // that share the z-stage operands of (q, k1, k2), each summed over g3 in
                // the same order as below (p <= 3)
                for (int t = tid; t < p1 * p1 * p1 * p1; t += blockDim.x) {
                    const int k12 = t % (p1 * p1), q = t / (p1 * p1);
                    const int i2 = q % p1, i3 = q / p1;
                    const int k1 = k12 % p1, k2 = k12 / p1;
                    const int vq = (i2 * p1 + k1) * p1 + k2;
                    double zl[nq];
#pragma unroll
                    for (int g3 = 0; g3 < nq; ++g3) zl[g3] = sL[i3][g3] * sV[0][vq][g3] + sD[i3][g3] * sV[1][vq][g3];
                    const int irow = i1 + p1 * (i2 + p1 * i3);
                    double *dst = Er + (int64_t)(i1 + p1 * q) * ld + sblk * Np + k12;
#pragma unroll
                    for (int k3 = 0; k3 < p1; ++k3) {
                        const int k = k12 + p1 * p1 * k3;
                        double v = 0.0;
#pragma unroll
                        for (int g3 = 0; g3 < nq; ++g3) v += zl[g3] * sL[k3][g3];
                        if (faces) {
                            // face terms of the faces that both node i and node k lie on (ascending lf)
                            unsigned m = sNm[irow] & sNm[k];
                            while (m) {
                                const int lf = __builtin_ctz(m);
                                m &= m - 1;
                                v += sF[lf * p1 * p1 * p1 * p1 + sNa[lf][irow] * p1 * p1 + sNa[lf][k]];
                            }
                        }
                        __builtin_nontemporal_store(v, dst + p1 * p1 * k3);
                    }
                }
            } else {
                // one output per thread and pass (p = 4: 3125 outputs, 13 passes)
                for (int t = tid; t < p1 * p1 * Np; t += blockDim.x) {
                    const int k = t % Np, q = t / Np;
                    const int i2 = q % p1, i3 = q / p1;
                    const int k1 = k % p1, k2 = (k / p1) % p1, k3 = k / (p1 * p1);
                    const int vq = (i2 * p1 + k1) * p1 + k2;
                    double v = 0.0;
                    for (int g3 = 0; g3 < nq; ++g3)
                        v += (sL[i3][g3] * sV[0][vq][g3] + sD[i3][g3] * sV[1][vq][g3]) * sL[k3][g3];
                    if (faces) {
                        // face terms of the faces that both node i and node k lie on (ascending lf)
                        const int irow = i1 + p1 * (i2 + p1 * i3);
                        unsigned m = sNm[irow] & sNm[k];
                        while (m) {
                            const int lf = __builtin_ctz(m);
                            m &= m - 1;
                            v += sF[lf * p1 * p1 * p1 * p1 + sNa[lf][irow] * p1 * p1 + sNa[lf][k]];
                        }
                    }
                    __builtin_nontemporal_store(v, Er + (int64_t)(i1 + p1 * q) * ld + sblk * Np + k);
                }
            }
        }
    };

    if (qrow) {
        // zeros over all n interior columns first (16-byte stores; n = 20 N_p is even and
        // the rows start on 64 bytes), then the mass block and K_j (identical for every
        // component c) over their columns; volume_block begins with a barrier
        const v2d zero2 = {0.0, 0.0};
        for (int t = tid; t < Np * (n / 2); t += blockDim.x)
            __builtin_nontemporal_store(zero2, (v2d *)(Er + (int64_t)(t / (n / 2)) * ld + 2 * (t % (n / 2))));
        for (int kind = 0; kind < 2; ++kind) {
            __syncthreads();
            for (int t = tid; t < 4 * Nq; t += blockDim.x) {
                const int d = t / Nq, g = t % Nq;
                double v;
                if (kind == 0) v = (d == 0) ? vg[g] : 0.0;
                else v = (d == 0) ? 0.0 : vg[g] * vg[(1 + 3 * (d - 1) + jdir) * Nq + g];
                sC[d][g] = v;
            }
            volume_block(kind == 0 ? r : 15 + c, false);
        }
    } else {
        for (int sblk = ug * 20 / kUG; sblk < (ug + 1) * 20 / kUG; ++sblk) {
            const int slot = (sblk < 15) ? 5 + sblk : sblk - 15;
            __syncthreads();
            for (int t = tid; t < 4 * Nq; t += blockDim.x)
                sC[t / Nq][t % Nq] = qpe[(int64_t)(4 * (20 * c + sblk) + t / Nq) * Nq + t % Nq];
            // the block's face coefficients at each face's Gauss points
            for (int t = tid; t < 6 * kNqfFace; t += blockDim.x) {
                const int lf = t / kNqfFace, sq = t % kNqfFace;
                if (sq < sNqf[lf]) sCf[lf][sq] = qpe[sFbase[lf] + (int64_t)(25 * c + slot) * sNqf[lf] + sq];
            }
            __syncthreads();
            // face terms: F[a0 a1][b0 b1] = sum_s c(s) phi_a(s) phi_b(s) per face, two 1-D stages
            for (int t = tid; t < 6 * p1 * p1 * kNQ; t += blockDim.x) {
                const int lf = t / (p1 * p1 * kNQ), rem = t % (p1 * p1 * kNQ);
                const int a0 = rem / (p1 * kNQ), b0 = (rem / kNQ) % p1, s1 = rem % kNQ;
                const int nqf1 = sPf[lf] + 2;
                double v = 0.0;
                if (s1 < nqf1) {
                    const double *cf = sCf[lf];
                    for (int s0 = 0; s0 < nqf1; ++s0)
                        v += sLf[lf][a0 * nqf1 + s0] * sLf[lf][b0 * nqf1 + s0] * cf[s0 + nqf1 * s1];
                }
                sG[t] = P.dt * v;
            }
            __syncthreads();
            for (int t = tid; t < 6 * p1 * p1 * p1 * p1; t += blockDim.x) {
                const int lf = t / (p1 * p1 * p1 * p1), rem = t % (p1 * p1 * p1 * p1);
                const int b1 = rem % p1, b0 = (rem / p1) % p1, a1 = (rem / (p1 * p1)) % p1, a0 = rem / (p1 * p1 * p1);
                const int nqf1 = sPf[lf] + 2;
                const double *gg = sG + lf * p1 * p1 * kNQ + (a0 * p1 + b0) * kNQ;
                double v = 0.0;
                for (int s1 = 0; s1 < nqf1; ++s1) v += sLf[lf][a1 * nqf1 + s1] * sLf[lf][b1 * nqf1 + s1] * gg[s1];
                sF[t] = v;
            }
            volume_block(sblk, true);
        }
    }
    if (ug != 0) return;  // uniform per workgroup
    // ---- trace columns B: face by face, B_lf[cp][a0 a1][b0 b1] = sum_s c_cp(s) phi_a(s) mu_b(s)
    for (int lf = 0; lf < 6; ++lf) {
        const int pf1 = sPf[lf] + 1, nqf1 = sPf[lf] + 2, Nqf = sNqf[lf], Nfp = pf1 * pf1;
        __syncthreads();
        for (int t = tid; t < 5 * p1 * pf1 * nqf1; t += blockDim.x) {
            const int cp = t / (p1 * pf1 * nqf1), rem = t % (p1 * pf1 * nqf1);
            const int a0 = rem / (pf1 * nqf1), b0 = (rem / nqf1) % pf1, s1 = rem % nqf1;
            double v = 0.0;
            if (!qrow || cp == c) {
                const double *cf = qrow ? dm.fgeo + dm.fgeo_off[6 * e + lf] + (int64_t)jdir * Nqf
                                        : qpe + sFbase[lf] + (int64_t)(25 * c + 20 + cp) * Nqf;
                for (int s0 = 0; s0 < nqf1; ++s0)
                    v += sLf[lf][a0 * nqf1 + s0] * sMf[lf][b0 * nqf1 + s0] * cf[s0 + nqf1 * s1];
                v *= qrow ? -1.0 : P.dt;
            }
            sG[t] = v;
        }
        __syncthreads();
        for (int t = tid; t < 5 * p1 * p1 * Nfp; t += blockDim.x) {
            const int cp = t / (p1 * p1 * Nfp), rem = t % (p1 * p1 * Nfp);
            const int a = rem / Nfp, b = rem % Nfp;
            const int a0 = a / p1, a1 = a % p1, b0 = b % pf1, b1 = b / pf1;
            const double *gg = sG + (cp * p1 * pf1 + a0 * pf1 + b0) * nqf1;
            double v = 0.0;
            for (int s1 = 0; s1 < nqf1; ++s1) v += sLf[lf][a1 * nqf1 + s1] * sMf[lf][b1 * nqf1 + s1] * gg[s1];
            sF[t] = v;
        }
        __syncthreads();
        // a thread keeps one column (ncol = 5 N_fp <= 125) and walks rows; a row
        // off the face is zero, a row on it reads its face-local index a0 p1 + a1
        const int ncol = 5 * Nfp, groups = blockDim.x / ncol;
        if (tid < groups * ncol) {
            const int col = tid % ncol, cp = col / Nfp, b = col % Nfp;
            const double *fc = sF + cp * p1 * p1 * Nfp + b;
            double *dst = Er + n + toff[lf] + col;
            for (int i = tid / ncol; i < Np; i += groups)
                __builtin_nontemporal_store(((sNm[i] >> lf) & 1u) ? fc[sNa[lf][i] * Nfp] : 0.0, dst + (int64_t)i * ld);
        }
    }
    // ---- residual column and padding: the residual's point coefficients in LDS,
    // the sum over the Gauss points split over two halves of the threads
    __syncthreads();
    {
        const double *rc = qpe + (int64_t)kVJac * Nq + (int64_t)(4 * r) * Nq;
        for (int t = tid; t < 4 * Nq; t += blockDim.x) sC[t / Nq][t % Nq] = rc[t];
    }
    __syncthreads();
    static_assert(2 * Np <= 256, "two threads per row");
    if (tid < 2 * Np) {
        const int i = tid % Np, h = tid / Np;
        const int i1 = i % p1, i2 = (i / p1) % p1, i3 = i / (p1 * p1);
        double v = 0.0;
        for (int g = h * (Nq / 2); g < (h + 1) * (Nq / 2) + h * (Nq % 2); ++g) {
            const int g1 = g % nq, g2 = (g / nq) % nq, g3 = g / (nq * nq);
            const double l0 = sL[i1][g1], l1 = sL[i2][g2], l2 = sL[i3][g3];
            v += sC[0][g] * l0 * l1 * l2 + sC[1][g] * sD[i1][g1] * l1 * l2 + sC[2][g] * l0 * sD[i2][g2] * l2 +
                 sC[3][g] * l0 * l1 * sD[i3][g3];
        }
        sG[tid] = v;
    }
    __syncthreads();
    for (int i = tid; i < Np; i += blockDim.x) {
        double v = sG[i] + sG[Np + i];
        const int i1 = i % p1, i2 = (i / p1) % p1, i3 = i / (p1 * p1);
        for (int lf = 0; lf < 6; ++lf) {
            int a0, a1;
            if (!face_idx(i1, i2, i3, lf, a0, a1)) continue;
            const int Nqf = sNqf[lf], nqf1 = sPf[lf] + 2;
            const double *fb = qpe + sFbase[lf];
            const double *fgl = dm.fgeo + dm.fgeo_off[6 * e + lf];
            for (int s = 0; s < Nqf; ++s) {
                const double ph = sLf[lf][a0 * nqf1 + s % nqf1] * sLf[lf][a1 * nqf1 + s / nqf1];
                if (qrow) v -= fgl[jdir * Nqf + s] * fb[(135 + c) * Nqf + s] * ph;
                else v += P.dt * fb[(125 + c) * Nqf + s] * ph;
            }
        }
        Er[(int64_t)i * ld + n + f] = v;
        for (int64_t col = n + f + 1; col < ld; ++col) Er[(int64_t)i * ld + col] = 0.0;
    }
}

// Trace rows of local face lf: [C | D | R_uh] rows of this element's side, one
// workgroup per (face, element): the numerical flux on an interior face, the
// boundary residual on a boundary face.  Only the columns of the face's own
// nodes (C), of the face's trace block (D) and the residual column are
// nonzero.  Rows go component by component (c = row / N_fp), kTR rows per
// pass.  In a pass each thread takes one (row, slot) pair (slots 0..19: C by
// column field, 20..24: D by trace component, 25: the residual column), forms
// its weights w(s) = coefficient(c, slot)(s) mu_a(s) at the face's Gauss
// points in registers and all of the pair's entries as dot products over the
// Gauss points with phi_k(s) (C) or mu_b(s) (D), into a compact LDS row; a
// column map then writes every row in one coalesced sweep, zeros included.
constexpr int kTR = 8;                              // trace rows per pass
constexpr int kNqfMax = kNQ * kNQ, kNfpMax = kP1 * kP1;
constexpr int kLdMax = (20 * kP1 * kP1 * kP1 + 30 * kNfpMax + 1 + 7) / 8 * 8;
constexpr int kTOut = 20 * kNfpMax + 5 * kNfpMax + 1;  // nonzero entries of a trace row, at most

__global__ void __launch_bounds__(256) k_assemble_trace_rows(DevMesh dm, Phys P, int e0, const double *__restrict__ qp,
                                                             double *__restrict__ Ebase) {
    const int e = e0 + blockIdx.y, lf = blockIdx.x;
    const int p = dm.elem_p[e], p1 = p + 1, Np = p1 * p1 * p1, nq = p + 2, Nq = nq * nq * nq;
    const int *toff = dm.toff + 7 * e;
    const int n = 20 * Np, f = toff[6];
    const int ld = (int)e_ld(n, f);
    double *E = Ebase + (dm.E_off[e] - dm.E_off[e0]);
    const double *qpe = qp + (dm.qp_off[e] - dm.qp_off[e0]);
    const int tid = threadIdx.x;
    __shared__ double sLf[6][30], sMf[6][30];
    __shared__ int sPf[6], sNqf[6];
    __shared__ int64_t sFbase[6];
    __shared__ double sPhi[kNfpMax][kNqfMax], sMu[kNfpMax][kNqfMax];
    __shared__ double sK[26][kNqfMax];  // coefficients of the current component c
    __shared__ double sOut[kTR][kTOut];  // the nonzero entries of the pass's rows
    __shared__ int sMap[kLdMax];         // column -> index into a row of sOut, or -1
    load_face_tables(dm, e, p, Nq, sLf, sMf, sPf, sNqf, sFbase);
    __syncthreads();
    const int pf1 = sPf[lf] + 1, nqf1 = pf1 + 1, Nfp = pf1 * pf1, Nqf = sNqf[lf];
    const int F = dm.elem_face[6 * e + lf], bc = dm.face_bc[F];
    const double *fb = qpe + sFbase[lf];
    double *Et = E + (int64_t)(n + toff[lf]) * ld;
    const int nC = 20 * p1 * p1;  // C entries of a row: column field x, face node y at x p1^2 + y
    // element basis phi_k and trace basis mu_b at the face's Gauss points
    for (int t = tid; t < kNfpMax * Nqf; t += blockDim.x) {
        const int k = t / Nqf, sq = t % Nqf, s0 = sq % nqf1, s1 = sq / nqf1;
        sPhi[k][sq] = (k < p1 * p1) ? sLf[lf][(k % p1) * nqf1 + s0] * sLf[lf][(k / p1) * nqf1 + s1] : 0.0;
        sMu[k][sq] = (k < Nfp) ? sMf[lf][(k % pf1) * nqf1 + s0] * sMf[lf][(k / pf1) * nqf1 + s1] : 0.0;
    }
    for (int col = tid; col < ld; col += blockDim.x) {
        int idx = -1;
        if (col < n) {
            const int sblk = col / Np, k = col % Np;
            int ka0, ka1;
            if (on_face(k, p1, lf, ka0, ka1)) {
                const int slot = (sblk < 15) ? 5 + sblk : sblk - 15;
                idx = slot * p1 * p1 + ka0 + p1 * ka1;
            }
        } else if (col < n + f) {
            const int cc = col - n;
            if (cc >= toff[lf] && cc < toff[lf + 1]) idx = nC + (cc - toff[lf]);
        } else if (col == n + f) {
            idx = nC + 5 * Nfp;
        }
        sMap[col] = idx;
    }
    const int rr_t = tid / 26, slot_t = tid % 26;  // this thread's (row of the pass, slot)
    for (int c = 0; c < 5; ++c) {
        __syncthreads();
        for (int t = tid; t < 26 * Nqf; t += blockDim.x) {
            const int slot = t / Nqf, sq = t % Nqf;
            sK[slot][sq] = (slot == 25) ? fb[(int64_t)((bc ? 130 : 125) + c) * Nqf + sq]
                                        : fb[(int64_t)((bc ? 140 : 0) + 25 * c + slot) * Nqf + sq];
        }
        for (int a0 = 0; a0 < Nfp; a0 += kTR) {
            const int nr = min(kTR, Nfp - a0);
            __syncthreads();  // sK ready; the previous pass's sweep is done with sOut
            if (rr_t < nr) {
                const int a = a0 + rr_t;  // trace row c Nfp + a tests mu_a
                double w[kNqfMax];
#pragma unroll
                for (int sq = 0; sq < kNqfMax; ++sq) w[sq] = sq < Nqf ? sK[slot_t][sq] * sMu[a][sq] : 0.0;
                double *out = sOut[rr_t];
                if (slot_t == 25) {
                    double v = 0.0;
#pragma unroll
                    for (int sq = 0; sq < kNqfMax; ++sq)
                        if (sq < Nqf) v += w[sq];
                    out[nC + 5 * Nfp] = v;
                } else {
                    const bool isC = slot_t < 20;
                    const int ny = isC ? p1 * p1 : Nfp;
                    double *o = isC ? out + slot_t * p1 * p1 : out + nC + (slot_t - 20) * Nfp;
                    for (int y = 0; y < ny; ++y) {
                        const double *brow = isC ? sPhi[y] : sMu[y];
                        double v = 0.0;
#pragma unroll
                        for (int sq = 0; sq < kNqfMax; ++sq)
                            if (sq < Nqf) v += w[sq] * brow[sq];
                        o[y] = v;
                    }
                }
            }
            __syncthreads();
            for (int rr = 0; rr < nr; ++rr) {
                double *dst = Et + (int64_t)(c * Nfp + a0 + rr) * ld;
                const double *out = sOut[rr];
                for (int c2 = tid; c2 < ld / 2; c2 += blockDim.x) {  // ld and the row starts are multiples of 8
                    const int i0 = sMap[2 * c2], i1 = sMap[2 * c2 + 1];
                    const v2d v = {i0 >= 0 ? out[i0] : 0.0, i1 >= 0 ? out[i1] : 0.0};
                    __builtin_nontemporal_store(v, (v2d *)(dst + 2 * c2));
                }
            }
        }
    }
}

}  // namespace

int launch_element_system(const hdg_ctx *ctx, int e0, int ne, const double *Q, const double *U,
                          const double *Un, const double *Uhat, const double *nu, const double *Ub,
                          double *E, double *qp, hipStream_t s) {
    const DevMesh &dm = ctx->dm;
    const Phys P = ctx->phys;
    hipLaunchKernelGGL(k_qp_volume, dim3(ne), dim3(256), 0, s, dm, P, e0, Q, U, Un, nu, qp);
    hipLaunchKernelGGL(k_qp_face, dim3(6, ne), dim3(64), 0, s, dm, P, e0, Q, U, Uhat, nu, Ub, qp);
    const double *qpc = qp;
    unsigned degrees = 0;
    for (int e = e0; e < e0 + ne; ++e) degrees |= 1u << ctx->elem_p[e];
    if (degrees & 2u) hipLaunchKernelGGL(k_assemble_field_rows<1>, dim3(15 + 5 * kUG, ne), dim3(256), 0, s, dm, P, e0, qpc, E);
    if (degrees & 4u) hipLaunchKernelGGL(k_assemble_field_rows<2>, dim3(15 + 5 * kUG, ne), dim3(256), 0, s, dm, P, e0, qpc, E);
    if (degrees & 8u) hipLaunchKernelGGL(k_assemble_field_rows<3>, dim3(15 + 5 * kUG, ne), dim3(256), 0, s, dm, P, e0, qpc, E);
    if (degrees & 16u) hipLaunchKernelGGL(k_assemble_field_rows<4>, dim3(15 + 5 * kUG, ne), dim3(256), 0, s, dm, P, e0, qpc, E);
    hipLaunchKernelGGL(k_assemble_trace_rows, dim3(6, ne), dim3(256), 0, s, dm, P, e0, qpc, E);
    return (int)hipGetLastError();
}

}  // namespace hdg
