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
// Per panel of kNB columns (all elements of a chunk advance together):
//   k_panel      one workgroup per element: factor the panel (16-column
//                sub-panels held in registers), intra-panel updates, record
//                the row permutation of the panel
//   k_swap_trsm  every trailing column: apply the permutation, then
//                U12 = L11^{-1} A12 (unit lower triangular solve)
//   k_update     A22 -= L21 U12 with FP64 MFMA (16x16x4), 128x128 tiles,
//                tiles of one element kept on one XCD (shared L2)
// then k_extract copies [S^K | g^K] out (column-major).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "hdg_internal.h"

namespace hdg {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kNB = 64;       // panel width
constexpr int kW = 16;        // register sub-panel width
constexpr int kPT = 512;      // panel kernel threads
constexpr int kPermMax = 2 * kNB;
// per element, per panel step: [0] = number of displaced rows,
// [1 .. kNB] source row of each top row, then (dst, src) pairs of displaced rows
constexpr int kPermInts = 1 + kNB + 2 * kNB;

struct ElemDims {
    int n, f, mrows;  // mrows = n + f
    int64_t ld;
};
// Bordered systems factored here: mode 0 = element systems (n = 20 N_p, f = f_e),
// mode 1 = Schwarz inversion systems [[S_r, I], [I, 0]] (n = f = f_r).
struct SysDesc {
    int mode;
    const int64_t *off;  // [n_elem+1] offsets (doubles) of the systems
};
__device__ inline ElemDims elem_dims(const DevMesh &dm, const SysDesc &sd, int e) {
    ElemDims d;
    if (sd.mode == 0) {
        const int p = dm.elem_p[e];
        d.n = 20 * (p + 1) * (p + 1) * (p + 1);
    } else {
        d.n = dm.toff[7 * e + 6];
    }
    d.f = dm.toff[7 * e + 6];
    d.mrows = d.n + d.f;
    d.ld = e_ld(d.n, d.f);
    return d;
}

__device__ inline void argmax_combine(double &v, int &r, double v2, int r2) {
    if (v2 > v || (v2 == v && r2 < r)) { v = v2; r = r2; }
}

// Compute the net row permutation of a sequence of swaps (row base+jj <-> piv[jj]).
// Produces for each top row its source row, and (dst, src) for rows outside the top block.
__device__ void build_perm(int base, int w, const int *piv, int *top_src, int *ndisp, int *disp, int *rows,
                           int *cont) {
    int cnt = 0;
    for (int jj = 0; jj < w; ++jj) { rows[cnt] = base + jj; cont[cnt] = base + jj; ++cnt; }
    for (int jj = 0; jj < w; ++jj) {
        const int a = base + jj, b = piv[jj];
        if (a == b) continue;
        int ia = -1, ib = -1;
        for (int t = 0; t < cnt; ++t) {
            if (rows[t] == a) ia = t;
            if (rows[t] == b) ib = t;
        }
        if (ib < 0) { rows[cnt] = b; cont[cnt] = b; ib = cnt++; }
        const int tmp = cont[ia];
        cont[ia] = cont[ib];
        cont[ib] = tmp;
    }
    for (int jj = 0; jj < w; ++jj) top_src[jj] = cont[jj];
    int nd = 0;
    for (int t = w; t < cnt; ++t)
        if (cont[t] != rows[t]) { disp[2 * nd] = rows[t]; disp[2 * nd + 1] = cont[t]; ++nd; }
    *ndisp = nd;
}

// ------------------------------------------------------------------ panel
template <int R>
__global__ void __launch_bounds__(kPT) k_panel(DevMesh dm, SysDesc sd, int e0, int k0, double *__restrict__ Ebase,
                                               int *__restrict__ perm_all, double *__restrict__ linv_all,
                                               int *__restrict__ info) {
    const int e = e0 + blockIdx.x;
    const ElemDims dd = elem_dims(dm, sd, e);
    if (k0 >= dd.n) return;
    const int nb = min(kNB, dd.n - k0);
    double *E = Ebase + (sd.off[e] - sd.off[e0]);
    const int64_t ld = dd.ld;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    __shared__ double s_val[kPT / 64];
    __shared__ int s_row[kPT / 64];
    __shared__ double s_prow[kW], s_krow[kW];
    __shared__ int s_pr, s_bad;
    __shared__ int s_piv[kNB];
    __shared__ int s_top[kNB], s_disp[2 * kNB], s_nd;
    __shared__ double s_L[kW][kW];
    __shared__ double s_U[kW][kNB];
    __shared__ int s_rows[2 * kNB], s_cont[2 * kNB];
    __shared__ double s_Lf[kNB][kNB + 1], s_Li[kNB][kNB + 1];
    int info_k = 0;

    for (int j0 = 0; j0 < nb; j0 += kW) {
        const int w = min(kW, nb - j0), cb = k0 + j0;
        double a[R][kW];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int r = cb + tid + kPT * i;
#pragma unroll
            for (int c = 0; c < kW; ++c) a[i][c] = (r < dd.mrows && c < w) ? E[(int64_t)r * ld + cb + c] : 0.0;
        }
        for (int jj = 0; jj < w; ++jj) {
            const int k = cb + jj;
            double best = -1.0;
            int brow = INT_MAX;
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int r = cb + tid + kPT * i;
                if (r >= k && r < dd.n) {
                    double v = 0.0;
#pragma unroll
                    for (int c = 0; c < kW; ++c)
                        if (c == jj) v = fabs(a[i][c]);
                    if (!(v == v)) v = INFINITY;  // a NaN pivot candidate is reported below
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
            if (tid == 0) {
                double b = s_val[0];
                int br = s_row[0];
                for (int t = 1; t < kPT / 64; ++t) argmax_combine(b, br, s_val[t], s_row[t]);
                const bool bad = !(b > 0.0) || !(b < INFINITY) || br == INT_MAX;
                s_bad = bad;
                s_pr = bad ? k : br;
                s_piv[j0 + jj] = s_pr;
            }
            __syncthreads();
            const int pr = s_pr;
            if (s_bad && info_k == 0) info_k = k + 1;
            // exchange rows k and pr through LDS
            const int ok_ = k - cb, opr = pr - cb;
            if (tid == opr % kPT) {
#pragma unroll
                for (int i = 0; i < R; ++i)
                    if (i == opr / kPT)
#pragma unroll
                        for (int c = 0; c < kW; ++c) s_prow[c] = a[i][c];
            }
            if (tid == ok_ % kPT) {
#pragma unroll
                for (int i = 0; i < R; ++i)
                    if (i == ok_ / kPT)
#pragma unroll
                        for (int c = 0; c < kW; ++c) s_krow[c] = a[i][c];
            }
            __syncthreads();
            if (pr != k) {
                if (tid == ok_ % kPT) {
#pragma unroll
                    for (int i = 0; i < R; ++i)
                        if (i == ok_ / kPT)
#pragma unroll
                            for (int c = 0; c < kW; ++c) a[i][c] = s_prow[c];
                }
                if (tid == opr % kPT) {
#pragma unroll
                    for (int i = 0; i < R; ++i)
                        if (i == opr / kPT)
#pragma unroll
                            for (int c = 0; c < kW; ++c) a[i][c] = s_krow[c];
                }
            }
            double pv = 0.0;
#pragma unroll
            for (int c = 0; c < kW; ++c)
                if (c == jj) pv = s_prow[c];
            const bool bad = s_bad;
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int r = cb + tid + kPT * i;
                if (r > k && r < dd.mrows) {
                    double l = 0.0;
#pragma unroll
                    for (int c = 0; c < kW; ++c)
                        if (c == jj) l = bad ? 0.0 : a[i][c] / pv;
#pragma unroll
                    for (int c = 0; c < kW; ++c) {
                        if (c == jj) a[i][c] = l;
                        else if (c > jj) a[i][c] -= l * s_prow[c];
                    }
                }
            }
            __syncthreads();
        }
        // write the factored sub-panel back; keep L11 of the sub-panel in LDS
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int r = cb + tid + kPT * i;
            if (r < dd.mrows)
#pragma unroll
                for (int c = 0; c < kW; ++c)
                    if (c < w) E[(int64_t)r * ld + cb + c] = a[i][c];
            if (i == 0 && tid < kW)
#pragma unroll
                for (int c = 0; c < kW; ++c) s_L[tid][c] = a[0][c];
        }
        if (tid == 0) build_perm(cb, w, s_piv + j0, s_top, &s_nd, s_disp, s_rows, s_cont);
        __syncthreads();
        // apply the sub-panel's row permutation to the other panel columns
        // (left: earlier sub-panels' L; right: not yet factored columns)
        const int nleft = j0, nright = nb - j0 - w, nother = nleft + nright;
        {
            // phase 1: read new values of the top rows and of the displaced rows
            const int nd = s_nd;
            const int items = (w + nd) * nother;  // <= 32 * 48 < 4 * kPT
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
                for (int r = 0; r < kW; ++r)
                    if (r < w) {
                        E[(int64_t)(cb + r) * ld + col] = x[r];
                        s_U[r][cidx] = x[r];
                    } else {
                        s_U[r][cidx] = 0.0;
                    }
            }
            __syncthreads();
            // rows below the sub-panel: E[r][right] -= L[r][0:w] U[0:w][right]
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int r = cb + tid + kPT * i;
                if (r < cb + w || r >= dd.mrows) continue;
                double *row = E + (int64_t)r * ld + cb + w;
                for (int cidx = 0; cidx < nright; ++cidx) {
                    double v = row[cidx];
#pragma unroll
                    for (int jj = 0; jj < kW; ++jj) v -= a[i][jj] * s_U[jj][cidx];
                    row[cidx] = v;
                }
            }
            __syncthreads();
        }
    }
    // the permutation of the whole panel, for the trailing columns
    int *pm = perm_all + (int64_t)blockIdx.x * kPermInts;
    if (tid == 0) {
        int nd;
        build_perm(k0, nb, s_piv, pm + 1, &nd, pm + 1 + kNB, s_rows, s_cont);
        pm[0] = nd;
    }
    // L11^{-1} (unit lower, nb x nb embedded in kNB x kNB) for the trailing columns
    for (int t = tid; t < kNB * kNB; t += kPT) {
        const int r = t / kNB, c = t % kNB;
        s_Lf[r][c] = (r < nb && c < r) ? E[(int64_t)(k0 + r) * ld + k0 + c] : 0.0;
    }
    __syncthreads();
    if (tid < kNB) {
        const int j = tid;
        for (int r = 0; r < kNB; ++r) {
            double x = (r == j) ? 1.0 : 0.0;
            if (r > j)
                for (int rr = j; rr < r; ++rr) x -= s_Lf[r][rr] * s_Li[rr][j];
            s_Li[r][j] = (r < nb) ? x : 0.0;
        }
    }
    __syncthreads();
    double *li = linv_all + (int64_t)blockIdx.x * kNB * kNB;
    for (int t = tid; t < kNB * kNB; t += kPT) li[t] = s_Li[t / kNB][t % kNB];
    if (tid == 0 && info_k && info[e] == 0) info[e] = info_k;
}

// ------------------------------------------------------------ swap + trsm
// For a tile of 64 trailing columns: gather the permuted top rows, move the
// displaced rows, and form U12 = L11^{-1} (P A12) with FP64 MFMA.
__global__ void __launch_bounds__(256) k_swap_trsm(DevMesh dm, SysDesc sd, int e0, int k0, double *__restrict__ Ebase,
                                                   const int *__restrict__ perm_all,
                                                   const double *__restrict__ linv_all) {
    const int e = e0 + blockIdx.y;
    const ElemDims dd = elem_dims(dm, sd, e);
    if (k0 >= dd.n) return;
    const int nb = min(kNB, dd.n - k0);
    const int c0 = k0 + nb + blockIdx.x * 64, cend = dd.mrows + 1;
    if (c0 >= cend) return;  // uniform per block
    double *E = Ebase + (sd.off[e] - sd.off[e0]);
    const int64_t ld = dd.ld;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    __shared__ double sA[kNB][64 + 1];
    __shared__ double sLi[kNB][kNB + 1];
    __shared__ int sperm[kPermInts];
    const int *pm = perm_all + (int64_t)blockIdx.y * kPermInts;
    for (int t = tid; t < kPermInts; t += 256) sperm[t] = pm[t];
    const double *li = linv_all + (int64_t)blockIdx.y * kNB * kNB;
    for (int t = tid; t < kNB * kNB; t += 256) sLi[t / kNB][t % kNB] = li[t];
    __syncthreads();
    for (int t = tid; t < kNB * 64; t += 256) {
        const int r = t / 64, c = t % 64;
        sA[r][c] = (r < nb && c0 + c < cend) ? E[(int64_t)sperm[1 + r] * ld + c0 + c] : 0.0;
    }
    const int nd = sperm[0];
    for (int t = tid; t < nd * 64; t += 256) {
        const int d = t / 64, c = t % 64;
        if (c0 + c < cend) {
            const int dst = sperm[1 + kNB + 2 * d], src = sperm[1 + kNB + 2 * d + 1];
            E[(int64_t)dst * ld + c0 + c] = E[(int64_t)src * ld + c0 + c];
        }
    }
    __syncthreads();
    // wave w: rows 16w .. 16w+15 of U12, all 64 columns (4 MFMA blocks)
    d4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = (d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < kNB; kk += 4) {
        const double a = sLi[16 * wave + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double b = sA[kk + (lane >> 4)][16 * j + (lane & 15)];
            acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
        }
    }
    // all reads of the top rows (sA) are done; write U12
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = 16 * wave + 4 * q + (lane >> 4), c = c0 + 16 * j + (lane & 15);
            if (r < nb && c < cend) E[(int64_t)(k0 + r) * ld + c] = acc[j][q];
        }
}

// --------------------------------------------------------- trailing update
constexpr int kTM = 128, kTN = 128, kKC = 16, kLdsPad = 8;

__global__ void __launch_bounds__(256) k_update(DevMesh dm, SysDesc sd, int e0, int ne, int k0, int tiles_m, int tiles_n,
                                                double *__restrict__ Ebase) {
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
    const int nb = min(kNB, dd.n - k0);
    const int r0 = k0 + nb + (t / tiles_n) * kTM, c0 = k0 + nb + (t % tiles_n) * kTN;
    const int rend = dd.mrows, cend = dd.mrows + 1;
    if (r0 >= rend || c0 >= cend) return;
    double *E = Ebase + (sd.off[e] - sd.off[e0]);
    const int64_t ld = dd.ld;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;  // wave sub-tile origin
    __shared__ double sA[2][kKC][kTM + kLdsPad];  // -L21 chunk, [k][row]
    __shared__ double sB[2][kKC][kTN + kLdsPad];  // U12 chunk,  [k][col]

    // accumulators = current A22 tile; lane l, slot j -> row 4j + l/16, col l%16
    d4 acc[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = r0 + wr + 16 * bi + 4 * j + (lane >> 4), c = c0 + wc + 16 * bj + (lane & 15);
                acc[bi][bj][j] = (r < rend && c < cend) ? E[(int64_t)r * ld + c] : 0.0;
            }
    // chunk loader: 128x16 of L21 and 16x128 of U12, 8 values each per thread
    auto load_chunk = [&](int kc, double *ra, double *rb) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int idx = tid + 256 * q;
            // A: row = idx / 16, k = idx % 16 (row-major reads along k)
            const int ar = idx / kKC, ak = idx % kKC;
            const int gr = r0 + ar, gk = kc + ak;
            ra[q] = (gr < rend && gk < nb) ? -E[(int64_t)gr * ld + k0 + gk] : 0.0;
            // B: k = idx / 128, col = idx % 128
            const int bk = idx / kTN, bc = idx % kTN;
            const int gk2 = kc + bk, gc = c0 + bc;
            rb[q] = (gk2 < nb && gc < cend) ? E[(int64_t)(k0 + gk2) * ld + gc] : 0.0;
        }
    };
    auto store_chunk = [&](int buf, const double *ra, const double *rb) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int idx = tid + 256 * q;
            sA[buf][idx % kKC][idx / kKC] = ra[q];
            sB[buf][idx / kTN][idx % kTN] = rb[q];
        }
    };
    double ra[8], rb[8];
    load_chunk(0, ra, rb);
    store_chunk(0, ra, rb);
    __syncthreads();
    const int nchunks = (nb + kKC - 1) / kKC;
    for (int ch = 0; ch < nchunks; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nchunks) load_chunk((ch + 1) * kKC, ra, rb);
#pragma unroll
        for (int kk = 0; kk < kKC; kk += 4) {
            double av[4], bv[4];
#pragma unroll
            for (int bi = 0; bi < 4; ++bi) av[bi] = sA[buf][kk + (lane >> 4)][wr + 16 * bi + (lane & 15)];
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
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = r0 + wr + 16 * bi + 4 * j + (lane >> 4), c = c0 + wc + 16 * bj + (lane & 15);
                if (r < rend && c < cend) E[(int64_t)r * ld + c] = acc[bi][bj][j];
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
static int run_bordered_lu(const hdg_ctx *ctx, const SysDesc &sd, int e0, int ne, double *E, int *info,
                           void *workv, int maxn, int maxm, hipStream_t s) {
    const DevMesh &dm = ctx->dm;
    double *linv = (double *)workv;
    int *work = (int *)((char *)workv + sizeof(double) * (size_t)ne * kNB * kNB);
    hipLaunchKernelGGL(k_zero_int, dim3((ne + 255) / 256), dim3(256), 0, s, info + e0, ne);
    const int R = (maxm + kPT - 1) / kPT;
    for (int k0 = 0; k0 < maxn; k0 += kNB) {
        if (R <= 1) hipLaunchKernelGGL(k_panel<1>, dim3(ne), dim3(kPT), 0, s, dm, sd, e0, k0, E, work, linv, info);
        else if (R <= 2) hipLaunchKernelGGL(k_panel<2>, dim3(ne), dim3(kPT), 0, s, dm, sd, e0, k0, E, work, linv, info);
        else if (R <= 4) hipLaunchKernelGGL(k_panel<4>, dim3(ne), dim3(kPT), 0, s, dm, sd, e0, k0, E, work, linv, info);
        else if (R <= 7) hipLaunchKernelGGL(k_panel<7>, dim3(ne), dim3(kPT), 0, s, dm, sd, e0, k0, E, work, linv, info);
        else return (int)hipErrorInvalidValue;
        // grids cover the largest trailing block of the chunk (an element whose panel is
        // narrower starts its trailing block earlier; over-cover by one panel width)
        const int ncol = maxm + 1 - k0;
        hipLaunchKernelGGL(k_swap_trsm, dim3((ncol + 63) / 64, ne), dim3(256), 0, s, dm, sd, e0, k0, E,
                           (const int *)work, (const double *)linv);
        const int mr = maxm - k0;
        const int tm = (mr + kTM - 1) / kTM, tn = (ncol + kTN - 1) / kTN;
        const int total = ne * tm * tn;
        const int grid = (total + 7) / 8 * 8;
        hipLaunchKernelGGL(k_update, dim3(grid), dim3(256), 0, s, dm, sd, e0, ne, k0, tm, tn, E);
    }
    return (int)hipGetLastError();
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
    int err = run_bordered_lu(ctx, sd, e0, ne, E, info, work, maxn, maxm, s);
    if (err) return err;
    hipLaunchKernelGGL(k_extract, dim3((maxf + 1 + 31) / 32, (maxf + 31) / 32, ne), dim3(256), 0, s, ctx->dm, sd,
                       e0, (const double *)E, SK);
    return (int)hipGetLastError();
}

size_t bordered_lu_work(const hdg_ctx *ctx, int ne) {
    (void)ctx;
    return sizeof(double) * (size_t)ne * kNB * kNB + sizeof(int) * (size_t)ne * kPermInts;
}

// Schwarz blocks: systems [[S_r, I], [I, 0]] in `sys` (offsets asmsys_off), eliminated
// over the first f_r columns; the trailing block is -S_r^{-1}.
int run_asm_inversion(const hdg_ctx *ctx, double *sys, int *info, void *iwork, hipStream_t s) {
    const SysDesc sd{1, ctx->dm.asmsys_off};
    const int maxf = ctx->max_f;
    return run_bordered_lu(ctx, sd, 0, ctx->n_elem, sys, info, iwork, maxf, 2 * maxf, s);
}

}  // namespace hdg
