// Static condensation of the element systems (eqs. local-elimination,
// schur-trace), FP64.
//
// E^K = [[A B R_qu],[C D R_uh]] (row-major) is reduced by a right-looking
// blocked LU with partial pivoting over the first n columns, pivots taken
// among the interior rows 0..n-1 only, the elimination carried through the
// trace rows and the right-hand columns.  After the n pivots the trailing
// block is D - C A^{-1} B (= S^K) next to R_uh - C A^{-1} R_qu (= -g^K), and
// rows 0..n-1 hold U and L^{-1} P [B | R_qu] for the recovery.
//
// Two-level blocking, all elements of a chunk advancing together.  Per block
// of kNBO = 128 pivot columns (two panels of kNB = 64):
//   k_panel      one workgroup per element factors a 64-column panel (8-column
//                sub-panels held in registers), records its pivots, the net row
//                permutation and L11^{-1}
//   k_rowperm    applies a recorded permutation to a range of columns and forms
//                U12 = L11^{-1} P A12 with FP64 MFMA (for the 128-row block:
//                U_a = La^{-1} X_a, X_b -= L_ba U_a, U_b = Lb^{-1} X_b)
//   k_update     A22 -= L21 U12 with FP64 MFMA (16x16x4): first over the second
//                panel's columns (K = 64), then over every trailing column with
//                K = 128, which halves the trailing-matrix traffic of a 64-wide
//                right-looking update; 128x128 tiles, the tiles of one element
//                on one XCD (shared L2)
// then k_extract copies [S^K | g^K] out (column-major).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "hdg_internal.h"

namespace hdg {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

constexpr int kNB = 64;       // panel width
constexpr int kNBO = 128;     // pivot columns per trailing update
constexpr int kW = 8;         // register sub-panel width
constexpr int kPT = 512;      // panel kernel threads
static_assert(kW >= 8 && kPT >= 2 * 64, "panel scratch and permutation assumptions");
// A recorded permutation of w swaps (row base+jj <-> piv[jj]): [0] = number of
// displaced rows, [1 .. W] source row of each top row, then (dst, src) pairs.
constexpr int kPerm64 = 1 + kNB + 2 * kNB;
constexpr int kPerm128 = 1 + kNBO + 2 * kNBO;
// Per-element workspace: doubles [4][64*64] (L^{-1}, U^{-1} of the two panels), then
// ints: piv[128] | perm of panel 0 | perm of panel 1 | perm of the 128 block.
constexpr int kWsDbl = 4 * kNB * kNB;  // L^{-1} of panels 0, 1, then U^{-1} of panels 0, 1
constexpr int kWsPiv = 0, kWsPerm0 = kNBO, kWsPerm1 = kWsPerm0 + kPerm64, kWsPerm128 = kWsPerm1 + kPerm64;
constexpr int kWsInt = kWsPerm128 + kPerm128;

struct ElemDims {
    int n, f, mrows;  // mrows = n + f
    int64_t ld;
};
// Bordered systems factored here: mode 0 = element systems (n = 20 N_p, f = f_e),
// mode 1 = Schwarz inversion systems [[S_r, I], [I, 0]] (n = f = f_r, rounded up to even).
struct SysDesc {
    int mode;
    const int64_t *off;  // [n_elem+1] offsets (doubles) of the systems
};
__device__ inline ElemDims elem_dims(const DevMesh &dm, const SysDesc &sd, int e) {
    ElemDims d;
    if (sd.mode == 0) {
        const int p = dm.elem_p[e];
        d.n = 20 * (p + 1) * (p + 1) * (p + 1);
        d.f = dm.toff[7 * e + 6];
    } else {
        // Schwarz system of an element with an odd f carries one extra decoupled
        // unknown, so that every panel width and column offset stays even
        const int f = dm.toff[7 * e + 6];
        d.n = f + (f & 1);
        d.f = d.n;
    }
    d.mrows = d.n + d.f;
    d.ld = e_ld(d.n, d.f);
    return d;
}

__device__ inline void argmax_combine(double &v, int &r, double v2, int r2) {
    if (v2 > v || (v2 == v && r2 < r)) { v = v2; r = r2; }
}

// Net row permutation of the swaps (row base+t <-> row piv[t]), t = 0 .. w-1, applied
// in order, with piv[t] >= base+t.  top_src[t] is the row whose content ends in row
// base+t; disp holds (dst, src) for every row >= base+w that a swap touched, in the
// order of its first swap, and *ndisp their count.  The content a displaced row ends
// with is always an original top row (a top row is final once its own swap is done),
// so the displaced copies never read a row that another copy writes.
// Every thread of the block calls it (w <= 128, at least 128 threads); piv is in LDS;
// the results are visible to the block after its next barrier.
__device__ void block_net_perm(int base, int w, const int *piv, int *top_src, int *ndisp, int *disp,
                               int *s_wcnt) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // undo the swaps from the last to the first to find where position x's content came from
    auto source = [&](int x) {
        for (int t = w - 1; t >= 0; --t) {
            const int pt = piv[t];
            x = (x == base + t) ? pt : ((x == pt) ? base + t : x);
        }
        return x;
    };
    bool keep = false;
    int y = 0, src = 0;
    if (tid < w) {
        top_src[tid] = source(base + tid);
        y = piv[tid];
        keep = y >= base + w;
        for (int t = 0; keep && t < tid; ++t) keep = piv[t] != y;  // first swap of row y only
        if (keep) {
            src = source(y);
            keep = src != y;
        }
    }
    const unsigned long long bal = __ballot(keep);
    if (lane == 0 && wave < 2) s_wcnt[wave] = __popcll(bal);
    __syncthreads();
    if (keep) {
        const int pos = (wave == 1 ? s_wcnt[0] : 0) + __popcll(bal & ((1ull << lane) - 1));
        disp[2 * pos] = y;
        disp[2 * pos + 1] = src;
    }
    if (tid == 0) *ndisp = s_wcnt[0] + s_wcnt[1];
}

// ------------------------------------------------------------------ panel
// Factor the panel columns [k0, k0+nb) over the pivot rows [k0, n) (the trace
// rows n.. get their multipliers from k_crows).  Rows are distributed over the
// threads (row cb + tid + kPT i), kW columns at a time held in registers.
template <int R, int TAG>
__global__ void __launch_bounds__(kPT) k_panel(DevMesh dm, SysDesc sd, int e0, int k0, int slot, int kbase,
                                               double *__restrict__ Ebase, double *__restrict__ wsd,
                                               int *__restrict__ wsi, int *__restrict__ info) {
    const int e = e0 + blockIdx.x;
    const ElemDims dd = elem_dims(dm, sd, e);
    if (k0 >= dd.n) return;
    const int nb = min(kNB, dd.n - k0);
    const int n = dd.n;
    double *E = Ebase + (sd.off[e] - sd.off[e0]);
    const int64_t ld = dd.ld;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    __shared__ double s_val[kPT / 64];
    __shared__ int s_row[kPT / 64];
    __shared__ double s_prow[kW], s_krow[kW];
    __shared__ int s_piv[kNBO];
    __shared__ int s_top[kNB], s_disp[2 * kNB], s_nd;
    __shared__ double s_L[kW][kW];
    __shared__ double s_U[kW][kNB];
    __shared__ int s_piv2[kNBO], s_wcnt[2];
    __shared__ double s_T[kNB][kNB + 1], s_I[kNB][kNB + 1];
    int info_k = 0;

    for (int j0 = 0; j0 < nb; j0 += kW) {
        const int w = min(kW, nb - j0), cb = k0 + j0;
        double a[R][kW];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int r = cb + tid + kPT * i;
            const double *src = E + (int64_t)min(r, n - 1) * ld + cb;
            if (w == kW) {
#pragma unroll
                for (int c = 0; c < kW; c += 2) {
                    const v2d v = *(const v2d *)(src + c);
                    a[i][c] = (r < n) ? v.x : 0.0;
                    a[i][c + 1] = (r < n) ? v.y : 0.0;
                }
            } else {
#pragma unroll
                for (int c = 0; c < kW; ++c) a[i][c] = (r < n && c < w) ? src[c] : 0.0;
            }
        }
#pragma unroll
        for (int jj = 0; jj < kW; ++jj) {
            if (jj < w) {  // uniform; keeps jj a compile-time register index
            const int k = cb + jj;
            // pivot: largest |a| over rows k..n-1 (smallest row index on ties); NaN wins
            double best = -1.0;
            int brow = INT_MAX;
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int r = cb + tid + kPT * i;
                if (r >= k && r < n) {
                    double v = fabs(a[i][jj]);
                    if (!(v == v)) v = INFINITY;
                    argmax_combine(best, brow, v, r);
                }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double v2 = __shfl_xor(best, off);
                const int r2 = __shfl_xor(brow, off);
                argmax_combine(best, brow, v2, r2);
            }
            if (lane == 0) { s_val[wave] = best; s_row[wave] = brow; }
            __syncthreads();
            double bv = s_val[0];
            int pr = s_row[0];
#pragma unroll
            for (int t = 1; t < kPT / 64; ++t) argmax_combine(bv, pr, s_val[t], s_row[t]);
            const bool bad = !(bv > 0.0) || !(bv < INFINITY) || pr == INT_MAX;
            if (bad) {
                pr = k;
                if (info_k == 0) info_k = k + 1;
            }
            if (tid == 0) s_piv[j0 + jj] = pr;
            // exchange rows k and pr through LDS
            const int ok_ = k - cb, opr = pr - cb;
            if (tid == opr % kPT) {
#pragma unroll
                for (int i = 0; i < R; ++i)
                    if (i == opr / kPT)
#pragma unroll
                        for (int c = 0; c < kW; ++c) s_prow[c] = a[i][c];
            }
            if (tid == ok_ && pr != k) {
#pragma unroll
                for (int c = 0; c < kW; ++c) s_krow[c] = a[0][c];
            }
            __syncthreads();
            if (pr != k) {
                if (tid == ok_) {
#pragma unroll
                    for (int c = 0; c < kW; ++c) a[0][c] = s_prow[c];
                }
                if (tid == opr % kPT) {
#pragma unroll
                    for (int i = 0; i < R; ++i)
                        if (i == opr / kPT)
#pragma unroll
                            for (int c = 0; c < kW; ++c) a[i][c] = s_krow[c];
                }
            }
            const double pinv = bad ? 0.0 : 1.0 / s_prow[jj];
            double prow[kW];
#pragma unroll
            for (int c = jj + 1; c < kW; ++c) prow[c] = s_prow[c];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int r = cb + tid + kPT * i;
                if (r > k && r < n) {
                    const double l = a[i][jj] * pinv;
                    a[i][jj] = l;
#pragma unroll
                    for (int c = jj + 1; c < kW; ++c) a[i][c] -= l * prow[c];
                }
            }
            }
        }
        // write the factored sub-panel back; keep its L11 in LDS
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int r = cb + tid + kPT * i;
            double *dst = E + (int64_t)r * ld + cb;
            if (r < n && w == kW) {
#pragma unroll
                for (int c = 0; c < kW; c += 2) *(v2d *)(dst + c) = (v2d){a[i][c], a[i][c + 1]};
            } else if (r < n) {
#pragma unroll
                for (int c = 0; c < kW; ++c)
                    if (c < w) dst[c] = a[i][c];
            }
        }
        if (tid < kW) {
#pragma unroll
            for (int c = 0; c < kW; ++c) s_L[tid][c] = a[0][c];
        }
        block_net_perm(cb, w, s_piv + j0, s_top, &s_nd, s_disp, s_wcnt);
        __syncthreads();
        // apply the sub-panel's row permutation to the other panel columns
        // (left: earlier sub-panels' L; right: not yet factored columns)
        const int nleft = j0, nright = nb - j0 - w, nother = nleft + nright;
        {
            const int nd = s_nd;
            const int items = (w + nd) * nother;  // <= 2 kW (kNB - kW) < 4 kPT
            double vals[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int t = tid + q * kPT;
                vals[q] = 0.0;
                if (t < items) {
                    const int ridx = t / nother, cidx = t % nother;
                    const int col = (cidx < nleft) ? k0 + cidx : cb + w + (cidx - nleft);
                    const int src = (ridx < w) ? s_top[ridx] : s_disp[2 * (ridx - w) + 1];
                    vals[q] = E[(int64_t)src * ld + col];
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int t = tid + q * kPT;
                if (t < items) {
                    const int ridx = t / nother, cidx = t % nother;
                    const int col = (cidx < nleft) ? k0 + cidx : cb + w + (cidx - nleft);
                    const int dst = (ridx < w) ? cb + ridx : s_disp[2 * (ridx - w)];
                    E[(int64_t)dst * ld + col] = vals[q];
                }
            }
            __syncthreads();
        }
        if (nright > 0) {
            // U of the sub-panel rows in the right columns: unit lower solve
            for (int cidx = tid; cidx < nright; cidx += kPT) {
                const int col = cb + w + cidx;
                double x[kW];
#pragma unroll
                for (int r = 0; r < kW; ++r) x[r] = (r < w) ? E[(int64_t)(cb + r) * ld + col] : 0.0;
#pragma unroll
                for (int r = 0; r < kW; ++r)
#pragma unroll
                    for (int rr = 0; rr < r; ++rr) x[r] -= s_L[r][rr] * x[rr];
#pragma unroll
                for (int r = 0; r < kW; ++r) {
                    if (r < w) E[(int64_t)(cb + r) * ld + col] = x[r];
                    s_U[r][cidx] = (r < w) ? x[r] : 0.0;
                }
            }
            __syncthreads();
            // pivot rows below the sub-panel: E[r][right] -= L[r][0:w] U[0:w][right]
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int r = cb + tid + kPT * i;
                if (r < cb + w || r >= n) continue;
                double *row = E + (int64_t)r * ld + cb + w;
                for (int c8 = 0; c8 < nright; c8 += 8) {
                    double v[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) v[q] = (c8 + q < nright) ? row[c8 + q] : 0.0;
#pragma unroll
                    for (int jj = 0; jj < kW; ++jj)
#pragma unroll
                        for (int q = 0; q < 8; ++q) v[q] -= a[i][jj] * s_U[jj][(c8 + q) & (kNB - 1)];
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        if (c8 + q < nright) row[c8 + q] = v[q];
                }
            }
            __syncthreads();
        }
    }
    // record pivots, the panel's net permutation, L11^{-1} and U11^{-1}
    int *wi = wsi + (int64_t)blockIdx.x * kWsInt;
    for (int t = tid; t < nb; t += kPT) wi[kWsPiv + slot * kNB + t] = s_piv[t];
    {
        int *pm = wi + (slot == 0 ? kWsPerm0 : kWsPerm1);
        block_net_perm(k0, nb, s_piv, pm + 1, pm, pm + 1 + kNB, s_wcnt);
    }
    // second panel of a 128-column block: the net permutation of all its swaps
    // (pivots of panel 0 come from the previous launch, those of panel 1 from LDS)
    if (slot == 1) {
        const int n0 = k0 - kbase, nbo = n0 + nb;
        for (int t = tid; t < nbo; t += kPT) s_piv2[t] = (t < n0) ? wi[kWsPiv + t] : s_piv[t - n0];
        __syncthreads();
        int *pm = wi + kWsPerm128;
        block_net_perm(kbase, nbo, s_piv2, pm + 1, pm, pm + 1 + kNBO, s_wcnt);
    }
    for (int t = tid; t < kNB * kNB; t += kPT) {
        const int r = t / kNB, c = t % kNB;
        s_T[r][c] = (r < nb && c < nb) ? E[(int64_t)(k0 + r) * ld + k0 + c] : 0.0;
        s_I[r][c] = 0.0;
    }
    __syncthreads();
    // Both inverses by 8 x 8 block substitution over the whole block: first the
    // diagonal blocks (one thread per column), then one block row at a time,
    // P = (off-diagonal part of the row) x (finished rows of the inverse) and
    // X_row = -X_diag P.  Rows and columns >= nb act as identity and are
    // returned as zero.
    double (*s_P)[kNB] = s_U;  // [8][64] partial products
    if (tid < kNB) {
        // diagonal block of L11^{-1}: forward substitution, unit diagonal
        const int j = tid, bi = j & ~7, jl = j & 7;
        double x[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            double v = (r == jl) ? 1.0 : 0.0;
#pragma unroll
            for (int c = 0; c < r; ++c) v -= s_T[bi + r][bi + c] * x[c];
            x[r] = (r >= jl) ? v : 0.0;
            s_I[bi + r][j] = x[r];
        }
    }
    __syncthreads();
    for (int bI = 8; bI < kNB; bI += 8) {
        const int i = tid & 7, j = tid >> 3;  // j < bI: columns left of the block row
        if (j < bI) {
            double v = 0.0;
            for (int k = j & ~7; k < bI; ++k) v += s_T[bI + i][k] * s_I[k][j];
            s_P[i][j] = v;
        }
        __syncthreads();
        if (j < bI) {
            double v = 0.0;
#pragma unroll
            for (int c = 0; c < 8; ++c) v -= s_I[bI + i][bI + c] * s_P[c][j];
            s_I[bI + i][j] = v;
        }
        __syncthreads();
    }
    double *li = wsd + (int64_t)blockIdx.x * kWsDbl + slot * kNB * kNB;
    for (int t = tid; t < kNB * kNB; t += kPT) {
        const int r = t / kNB, c = t % kNB;
        li[t] = (r < nb && c < nb) ? s_I[r][c] : 0.0;
    }
    __syncthreads();
    for (int t = tid; t < kNB * kNB; t += kPT) s_I[t / kNB][t % kNB] = 0.0;
    __syncthreads();
    if (tid < kNB) {
        // diagonal block of U11^{-1}: back substitution
        const int j = tid, bi = j & ~7, jl = j & 7;
        double x[8];
#pragma unroll
        for (int r = 7; r >= 0; --r) {
            double v = (r == jl) ? 1.0 : 0.0;
#pragma unroll
            for (int c = r + 1; c < 8; ++c) v -= s_T[bi + r][bi + c] * x[c];
            const double d = (bi + r < nb) ? s_T[bi + r][bi + r] : 1.0;
            x[r] = (r <= jl) ? v / d : 0.0;
            s_I[bi + r][j] = x[r];
        }
    }
    __syncthreads();
    for (int bI = kNB - 16; bI >= 0; bI -= 8) {
        const int i = tid & 7, j = bI + 8 + (tid >> 3);  // columns right of the block row
        if (j < kNB) {
            double v = 0.0;
            for (int k = bI + 8; k <= (j | 7); ++k) v += s_T[bI + i][k] * s_I[k][j];
            s_P[i][j] = v;
        }
        __syncthreads();
        if (j < kNB) {
            double v = 0.0;
#pragma unroll
            for (int c = 0; c < 8; ++c) v -= s_I[bI + i][bI + c] * s_P[c][j];
            s_I[bI + i][j] = v;
        }
        __syncthreads();
    }
    double *ui = wsd + (int64_t)blockIdx.x * kWsDbl + (2 + slot) * kNB * kNB;
    for (int t = tid; t < kNB * kNB; t += kPT) {
        const int r = t / kNB, c = t % kNB;
        ui[t] = (r < nb && c < nb) ? s_I[r][c] : 0.0;
    }
    if (tid == 0 && info_k && info[e] == 0) info[e] = info_k;
}

// Multipliers of the trace rows n..n+f-1 in the panel columns [kp, kp+nb):
// L_C = C_panel U11^{-1} (FP64 MFMA), one workgroup per 64 trace rows.
template <int TAG>
__global__ void __launch_bounds__(256) k_crows(DevMesh dm, SysDesc sd, int e0, int kp, int slot,
                                               double *__restrict__ Ebase, const double *__restrict__ wsd) {
    const int e = e0 + blockIdx.y;
    const ElemDims dd = elem_dims(dm, sd, e);
    if (kp >= dd.n) return;
    const int nb = min(kNB, dd.n - kp);
    const int r0 = dd.n + blockIdx.x * 64;
    if (r0 >= dd.mrows) return;
    double *E = Ebase + (sd.off[e] - sd.off[e0]);
    const int64_t ld = dd.ld;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    __shared__ double sX[64][65];
    __shared__ double sU[kNB][kNB + 1];
    const double *ui = wsd + (int64_t)blockIdx.y * kWsDbl + (2 + slot) * kNB * kNB;
    for (int t = tid; t < kNB * kNB; t += 256) sU[t >> 6][t & 63] = ui[t];
    for (int t = tid; t < 64 * 64; t += 256) {
        const int r = t >> 6, c = t & 63;
        sX[r][c] = (r0 + r < dd.mrows && c < nb) ? E[(int64_t)(r0 + r) * ld + kp + c] : 0.0;
    }
    __syncthreads();
    d4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int kk = 0; kk < kNB; kk += 4) {
        const double av = sX[16 * wave + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double bv = sU[kk + (lane >> 4)][16 * j + (lane & 15)];
            acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = r0 + 16 * wave + 4 * q + (lane >> 4), c = 16 * j + (lane & 15);
            if (r < dd.mrows && c < nb) E[(int64_t)r * ld + kp + c] = acc[j][q];
        }
}

// ------------------------------------------------------- row permutation
// MODE 0: rows base..base+63 <- permuted (panel `slot`), U = L^{-1} X, on
//         columns [k0 + K_e, k0 + min(CW, n_e - k0))  (CW = 0: to the end)
// MODE 1: permutation of panel 1 only, on the columns of panel 0 (its L)
// MODE 2: 128-row block: X = P A12 (net permutation of both panels),
//         U_a = La^{-1} X_a, X_b -= L_ba U_a, U_b = Lb^{-1} X_b, on the trailing columns
// One workgroup per (64-column tile, element).
__device__ inline void mfma_64x64(const double (*Ls)[kNB + 1], const double (*X)[65], d4 acc[4], int lane, int wave) {
    // acc (rows 16 wave .. +15, 64 columns) = Ls (64x64) * X (64 x 64)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int kk = 0; kk < kNB; kk += 4) {
        const double a = Ls[16 * wave + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double b = X[kk + (lane >> 4)][16 * j + (lane & 15)];
            acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
        }
    }
}

template <int MODE, int TAG>
__global__ void __launch_bounds__(256) k_rowperm(DevMesh dm, SysDesc sd, int e0, int k0, int CW,
                                                 double *__restrict__ Ebase, const double *__restrict__ wsd,
                                                 const int *__restrict__ wsi) {
    const int e = e0 + blockIdx.y;
    const ElemDims dd = elem_dims(dm, sd, e);
    if (k0 >= dd.n) return;
    const int rem = dd.n - k0;
    int c_begin, c_end, base, nrows, permoff;
    if (MODE == 0) {
        const int K = min(kNB, rem);
        c_begin = k0 + K;
        c_end = CW > 0 ? k0 + min(CW, rem) : dd.mrows + 1;
        base = k0; nrows = K; permoff = kWsPerm0;
    } else if (MODE == 1) {
        if (rem <= kNB) return;
        c_begin = k0;
        c_end = k0 + kNB;
        base = k0 + kNB; nrows = min(kNB, rem - kNB); permoff = kWsPerm1;
    } else {
        const int nbo = min(kNBO, rem);
        c_begin = k0 + nbo;
        c_end = dd.mrows + 1;
        base = k0; nrows = nbo; permoff = (nbo > kNB) ? kWsPerm128 : kWsPerm0;
    }
    const int c0 = c_begin + blockIdx.x * 64;
    if (c0 >= c_end) return;  // uniform per block
    double *E = Ebase + (sd.off[e] - sd.off[e0]);
    const int64_t ld = dd.ld;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    __shared__ double sX[kNBO][65];
    __shared__ double sM[kNB][kNB + 1];
    __shared__ int sperm[kPerm128];
    const int *wi = wsi + (int64_t)blockIdx.y * kWsInt;
    const int W = (permoff == kWsPerm128) ? kNBO : kNB;
    const int permlen = 1 + W + 2 * W;
    for (int t = tid; t < permlen; t += 256) sperm[t] = wi[permoff + t];
    __syncthreads();
    // gather the permuted top rows, then move the displaced rows
    for (int t = tid; t < nrows * 64; t += 256) {
        const int r = t >> 6, c = t & 63;
        sX[r][c] = (c0 + c < c_end) ? E[(int64_t)sperm[1 + r] * ld + c0 + c] : 0.0;
    }
    for (int t = tid; t < (kNBO - nrows) * 64; t += 256) sX[nrows + (t >> 6)][t & 63] = 0.0;
    // a top row's source may be a displaced row: its old content must be read
    // before the displaced copies overwrite it
    __syncthreads();
    // displaced rows take original top rows, which are rewritten only after the
    // next barrier
    const int nd = sperm[0];
    for (int t = tid; t < nd * 64; t += 256) {
        const int d = t >> 6, c = t & 63;
        if (c0 + c < c_end) {
            const int dst = sperm[1 + W + 2 * d], src = sperm[1 + W + 2 * d + 1];
            E[(int64_t)dst * ld + c0 + c] = E[(int64_t)src * ld + c0 + c];
        }
    }
    if (MODE == 1) __syncthreads();
    if (MODE != 1) {
        const double *la = wsd + (int64_t)blockIdx.y * kWsDbl;
        d4 acc[4];
        // U_a = La^{-1} X_a
        for (int t = tid; t < kNB * kNB; t += 256) sM[t >> 6][t & 63] = la[t];
        __syncthreads();
        mfma_64x64(sM, sX, acc, lane, wave);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) sX[16 * wave + 4 * q + (lane >> 4)][16 * j + (lane & 15)] = acc[j][q];
        if (nrows > kNB) {
            // X_b -= L_ba U_a   (L_ba: rows base+64.., columns base.. of E, already permuted)
            __syncthreads();
            for (int t = tid; t < kNB * kNB; t += 256) {
                const int r = t >> 6, c = t & 63;
                sM[r][c] = (kNB + r < nrows) ? E[(int64_t)(base + kNB + r) * ld + base + c] : 0.0;
            }
            __syncthreads();
            mfma_64x64(sM, sX, acc, lane, wave);
            __syncthreads();
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) sX[kNB + 16 * wave + 4 * q + (lane >> 4)][16 * j + (lane & 15)] -= acc[j][q];
            // U_b = Lb^{-1} X_b
            __syncthreads();
            for (int t = tid; t < kNB * kNB; t += 256) sM[t >> 6][t & 63] = la[kNB * kNB + t];
            __syncthreads();
            mfma_64x64(sM, (const double (*)[65])(&sX[kNB][0]), acc, lane, wave);
            __syncthreads();
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) sX[kNB + 16 * wave + 4 * q + (lane >> 4)][16 * j + (lane & 15)] = acc[j][q];
        }
        __syncthreads();
    }
    for (int t = tid; t < nrows * 64; t += 256) {
        const int r = t >> 6, c = t & 63;
        if (c0 + c < c_end) E[(int64_t)(base + r) * ld + c0 + c] = sX[r][c];
    }
}

// --------------------------------------------------------- trailing update
// A22 -= L21 U12 with L21 = E[rows, k0 .. k0+K), U12 = E[k0 .. k0+K, cols],
// K = min(KW, n_e - k0); rows [k0+K, n+f), columns [k0+K, k0+min(CW, n_e-k0))
// (CW > 0) or [k0+K, n+f+1).  128 x 128 tile per workgroup, K in chunks of 16
// double-buffered through LDS, FP64 MFMA into zero-initialised accumulators,
// the subtraction from A22 in the epilogue.
constexpr int kTM = 128, kTN = 128, kKC = 16;
constexpr int kSA = kKC + 2;    // LDS row stride of the L21 chunk (rows x k)
constexpr int kSB = kTN + 16;   // LDS row stride of the U12 chunk (k x columns)

template <int TAG>
__global__ void __launch_bounds__(256, 2) k_update(DevMesh dm, SysDesc sd, int e0, int ne, int k0, int KW, int CW,
                                                   int tiles_m, int tiles_n, double *__restrict__ Ebase) {
    // XCD-aware mapping: consecutive workgroups go round-robin over the 8 XCDs;
    // give each XCD a contiguous range of (element, tile) work items.
    const int total = ne * tiles_m * tiles_n;
    const int per_xcd = (total + 7) / 8;
    const int w = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (w >= total) return;
    const int el = w / (tiles_m * tiles_n), t = w % (tiles_m * tiles_n);
    const int e = e0 + el;
    const ElemDims dd = elem_dims(dm, sd, e);
    if (k0 >= dd.n) return;
    const int rem = dd.n - k0;
    const int K = min(KW, rem);
    const int r0 = k0 + K + (t / tiles_n) * kTM;
    const int c0 = k0 + K + (t % tiles_n) * kTN;
    const int rend = dd.mrows;
    const int cend = CW > 0 ? k0 + min(CW, rem) : dd.mrows + 1;
    if (r0 >= rend || c0 >= cend) return;
    double *E = Ebase + (sd.off[e] - sd.off[e0]);
    const int64_t ld = dd.ld;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;  // wave sub-tile origin
    __shared__ double sA[2][kTM][kSA];
    __shared__ double sB[2][kKC][kSB];
    // chunk loads with 16-byte accesses: L21 chunk (128 rows x 16 k): 8 lanes per
    // row segment of 128 bytes, rows 32q + tid/8; U12 chunk (16 k x 128 columns):
    // one wave per k-row of 1 KB, k-rows 4q + tid/64.  Out-of-range entries are
    // read from a clamped in-range address and replaced by 0 (no branches): K and
    // every column offset are even, and a row holds ld >= n+f+1 entries.
    const int ar = tid >> 3, ak = (tid & 7) * 2;
    const int bk = tid >> 6, bc = (tid & 63) * 2;
    const double *arow[4];
    bool aok[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int row = r0 + 32 * q + ar;
        aok[q] = row < rend;
        arow[q] = E + (int64_t)min(row, rend - 1) * ld + k0;
    }
    const int bcol = c0 + bc;
    const bool bok0 = bcol < cend, bok1 = bcol + 1 < cend;
    const int bcolc = min(bcol, (cend - 1) & ~1);
    auto load_chunk = [&](int kc, v2d *ra, v2d *rb) {
        const int gk = kc + ak;
        const int gkc = min(gk, (K - 1) & ~1);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const v2d v = *(const v2d *)(arow[q] + gkc);
            ra[q].x = (aok[q] && gk < K) ? v.x : 0.0;
            ra[q].y = (aok[q] && gk + 1 < K) ? v.y : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int gk2 = kc + 4 * q + bk;
            const bool k2ok = gk2 < K;
            const v2d v = *(const v2d *)(E + (int64_t)(k0 + min(gk2, K - 1)) * ld + bcolc);
            rb[q].x = (k2ok && bok0) ? v.x : 0.0;
            rb[q].y = (k2ok && bok1) ? v.y : 0.0;
        }
    };
    auto store_chunk = [&](int buf, const v2d *ra, const v2d *rb) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            *(v2d *)&sA[buf][32 * q + ar][ak] = ra[q];
            *(v2d *)&sB[buf][4 * q + bk][bc] = rb[q];
        }
    };
    d4 acc[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = (d4){0.0, 0.0, 0.0, 0.0};
    v2d ra[4], rb[4];
    load_chunk(0, ra, rb);
    store_chunk(0, ra, rb);
    __syncthreads();
    const int nchunks = (K + kKC - 1) / kKC;
    for (int ch = 0; ch < nchunks; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nchunks) load_chunk((ch + 1) * kKC, ra, rb);
#pragma unroll
        for (int kk = 0; kk < kKC; kk += 4) {
            double av[4], bv[4];
#pragma unroll
            for (int bi = 0; bi < 4; ++bi) av[bi] = sA[buf][wr + 16 * bi + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) bv[bj] = sB[buf][kk + (lane >> 4)][wc + 16 * bj + (lane & 15)];
#pragma unroll
            for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                for (int bj = 0; bj < 4; ++bj)
                    acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[bi], bv[bj], acc[bi][bj], 0, 0, 0);
        }
        if (ch + 1 < nchunks) {
            store_chunk(buf ^ 1, ra, rb);
            __syncthreads();
        }
    }
    // epilogue: A22 -= product.  lane l, slot j -> row 4j + l/16, column l%16 of the 16x16 block
    const bool full = (r0 + kTM <= rend) && (c0 + kTN <= cend);
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = r0 + wr + 16 * bi + 4 * j + (lane >> 4);
            double *row = E + (int64_t)r * ld + c0 + wc + (lane & 15);
            if (full) {
#pragma unroll
                for (int bj = 0; bj < 4; ++bj) row[16 * bj] -= acc[bi][bj][j];
            } else if (r < rend) {
#pragma unroll
                for (int bj = 0; bj < 4; ++bj)
                    if (c0 + wc + 16 * bj + (lane & 15) < cend) row[16 * bj] -= acc[bi][bj][j];
            }
        }
}

// ------------------------------------------------------------------ extract
// SK (column-major f x (f+1)) = [ trailing f x f block | - last column ]
__global__ void __launch_bounds__(256) k_extract(DevMesh dm, SysDesc sd, int e0, const double *__restrict__ Ebase,
                                                 double *__restrict__ SK) {
    const int e = e0 + blockIdx.z;
    const ElemDims dd = elem_dims(dm, sd, e);
    const int f = dd.f;
    const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 32;  // i: row of S, j: column (0..f)
    if (i0 >= f || j0 > f) return;
    const double *E = Ebase + (sd.off[e] - sd.off[e0]);
    double *out = SK + dm.SK_off[e];
    __shared__ double tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int i = i0 + r, j = j0 + tx;
        double v = 0.0;
        if (i < f && j <= f) {
            v = E[(int64_t)(dd.n + i) * dd.ld + dd.n + j];
            if (j == f) v = -v;
        }
        tile[r][tx] = v;
    }
    __syncthreads();
    for (int c = ty; c < 32; c += 8) {
        const int j = j0 + c, i = i0 + tx;
        if (i < f && j <= f) out[(int64_t)j * f + i] = tile[tx][c];
    }
}

__global__ void k_zero_int(int *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

}  // namespace

// Run the bordered elimination on systems e0..e0+ne-1 described by sd.
template <int TAG>
static int run_bordered_lu_t(const hdg_ctx *ctx, const SysDesc &sd, int e0, int ne, double *E, int *info,
                             void *workv, int maxn, int maxm, int maxf_rows, hipStream_t s) {
    const DevMesh &dm = ctx->dm;
    double *wsd = (double *)workv;
    int *wsi = (int *)((char *)workv + sizeof(double) * (size_t)ne * kWsDbl);
    hipLaunchKernelGGL(k_zero_int, dim3((ne + 255) / 256), dim3(256), 0, s, info + e0, ne);
    const int R = (maxn + kPT - 1) / kPT;
    auto crows = [&](int kp, int slot) {
        if (maxf_rows > 0)
            hipLaunchKernelGGL((k_crows<TAG>), dim3((maxf_rows + 63) / 64, ne), dim3(256), 0, s, dm, sd, e0, kp, slot, E,
                               (const double *)wsd);
    };
    auto panel = [&](int k0, int slot, int kbase) {
        if (R <= 1) hipLaunchKernelGGL((k_panel<1, TAG>), dim3(ne), dim3(kPT), 0, s, dm, sd, e0, k0, slot, kbase, E, wsd, wsi, info);
        else if (R <= 2) hipLaunchKernelGGL((k_panel<2, TAG>), dim3(ne), dim3(kPT), 0, s, dm, sd, e0, k0, slot, kbase, E, wsd, wsi, info);
        else if (R <= 3) hipLaunchKernelGGL((k_panel<3, TAG>), dim3(ne), dim3(kPT), 0, s, dm, sd, e0, k0, slot, kbase, E, wsd, wsi, info);
        else hipLaunchKernelGGL((k_panel<5, TAG>), dim3(ne), dim3(kPT), 0, s, dm, sd, e0, k0, slot, kbase, E, wsd, wsi, info);
        crows(k0, slot);
    };
    auto update = [&](int k0, int KW, int CW, int rows, int cols) {
        if (rows <= 0 || cols <= 0) return;
        const int tm = (rows + kTM - 1) / kTM, tn = (cols + kTN - 1) / kTN;
        const int total = ne * tm * tn;
        hipLaunchKernelGGL((k_update<TAG>), dim3((total + 7) / 8 * 8), dim3(256), 0, s, dm, sd, e0, ne, k0, KW, CW, tm,
                           tn, E);
    };
    if (R > 5) return (int)hipErrorInvalidValue;
    for (int k0 = 0; k0 < maxn; k0 += kNBO) {
        panel(k0, 0, k0);
        if (maxn - k0 > kNB) {
            // rest of the 128-column block, then its second panel
            hipLaunchKernelGGL((k_rowperm<0, TAG>), dim3(1, ne), dim3(256), 0, s, dm, sd, e0, k0, kNBO, E,
                               (const double *)wsd, (const int *)wsi);
            update(k0, kNB, kNBO, maxm - k0, kNB);
            panel(k0 + kNB, 1, k0);
            hipLaunchKernelGGL((k_rowperm<1, TAG>), dim3(1, ne), dim3(256), 0, s, dm, sd, e0, k0, 0, E,
                               (const double *)wsd, (const int *)wsi);
            // trailing columns: 128-row permutation + block solve, K = 128 update
            const int ncol = maxm + 1 - k0;
            hipLaunchKernelGGL((k_rowperm<2, TAG>), dim3((ncol + 63) / 64, ne), dim3(256), 0, s, dm, sd, e0, k0, 0,
                               E, (const double *)wsd, (const int *)wsi);
            update(k0, kNBO, 0, maxm - k0, ncol);
        } else {
            const int ncol = maxm + 1 - k0;
            hipLaunchKernelGGL((k_rowperm<0, TAG>), dim3((ncol + 63) / 64, ne), dim3(256), 0, s, dm, sd, e0, k0, 0,
                               E, (const double *)wsd, (const int *)wsi);
            update(k0, kNB, 0, maxm - k0, ncol);
        }
    }
    return (int)hipGetLastError();
}

static int run_bordered_lu(const hdg_ctx *ctx, const SysDesc &sd, int e0, int ne, double *E, int *info,
                           void *workv, int maxn, int maxm, int maxf_rows, hipStream_t s) {
    if (sd.mode == 0) return run_bordered_lu_t<0>(ctx, sd, e0, ne, E, info, workv, maxn, maxm, maxf_rows, s);
    return run_bordered_lu_t<1>(ctx, sd, e0, ne, E, info, workv, maxn, maxm, maxf_rows, s);
}

int launch_condense_fp64(const hdg_ctx *ctx, int e0, int ne, double *E, double *SK, int *info, void *work,
                         hipStream_t s) {
    int maxn = 0, maxm = 0, maxf = 0;
    for (int e = e0; e < e0 + ne; ++e) {
        maxn = std::max(maxn, ctx->elem_n[e]);
        maxm = std::max(maxm, ctx->elem_n[e] + ctx->elem_f[e]);
        maxf = std::max(maxf, ctx->elem_f[e]);
    }
    const SysDesc sd{0, ctx->dm.E_off};
    int err = run_bordered_lu(ctx, sd, e0, ne, E, info, work, maxn, maxm, maxf, s);
    if (err) return err;
    hipLaunchKernelGGL(k_extract, dim3((maxf + 1 + 31) / 32, (maxf + 31) / 32, ne), dim3(256), 0, s, ctx->dm, sd,
                       e0, (const double *)E, SK);
    return (int)hipGetLastError();
}

size_t bordered_lu_work(const hdg_ctx *ctx, int ne) {
    (void)ctx;
    return sizeof(double) * (size_t)ne * kWsDbl + sizeof(int) * (size_t)ne * kWsInt;
}

// Schwarz blocks: systems [[S_r, I], [I, 0]] in `sys` (offsets asmsys_off), eliminated
// over the first f_r columns; the trailing block is -S_r^{-1}.
int run_asm_inversion(const hdg_ctx *ctx, double *sys, int *info, void *iwork, hipStream_t s) {
    const SysDesc sd{1, ctx->dm.asmsys_off};
    const int maxf = ctx->max_f + (ctx->max_f & 1);
    return run_bordered_lu(ctx, sd, 0, ctx->n_elem, sys, info, iwork, maxf, 2 * maxf, maxf, s);
}

}  // namespace hdg
