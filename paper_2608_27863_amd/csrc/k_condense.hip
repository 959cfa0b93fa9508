// Static condensation of the element systems (eqs. local-elimination,
// schur-trace), in FP64 and in mixed precision.
//
// FP64.  E^K = [[A B R_qu],[C D R_uh]] (row-major) is reduced by a right-looking
// blocked LU with partial pivoting over the first n columns, pivots taken
// among the interior rows 0..n-1 only, the elimination carried through the
// trace rows and the right-hand columns.  After the n pivots the trailing
// block is D - C A^{-1} B (= S^K) next to R_uh - C A^{-1} R_qu (= -g^K), and
// rows 0..n-1 hold U and L^{-1} P [B | R_qu] for the recovery.
//
// Mixed.  The interior rows [A | B R_qu] are copied to FP32 and factorised by
// the same blocked LU in FP32 (FP32 matrix cores, FP32 accumulation); a blocked
// back substitution gives X_0 = A^{-1}[B | R_qu] in FP32.  Each refinement step
// forms R = [B | R_qu] - A X in FP64 from the untouched FP64 system, solves
// A d = R with the FP32 factors and adds d to X in FP64.  Finally
// [S^K | -g^K] = [D | R_uh] - C X is formed with FP64 matrix cores and X is
// stored in place of [B | R_qu] for the recovery.
//
// Two-level blocking, all elements of a chunk advancing together.  Per block
// of kNBO = 128 pivot columns (two panels of kNB = 64):
//   k_panel      one workgroup per element factors a 64-column panel (8-column
//                sub-panels held in registers) in two 32-column halves, records
//                its pivots, the net row permutation, L11^{-1} and U11^{-1}
//   k_half       the first half's update of the second half's columns
//   k_crows      multipliers of the trace rows, L_C = C_panel U11^{-1}
//   k_rowperm    within the block: applies panel a's permutation to panel b's
//                columns and forms its U rows; applies panel b's permutation
//                to panel a's L
//   k_inv128     the off-diagonal blocks of the 128-row triangles' inverses
//   k_blocku     other columns: the block's net row permutation and
//                U12 = L11^{-1} P A12 as one triangular product on matrix cores
//                (blocks go in pairs: the far columns get one K = 256 update)
//   k_update     A22 -= L21 U12 on matrix cores (16x16x4): over the second
//                panel's columns (K = 64), over the second block's columns
//                (K = 128), then over every column beyond the pair with K = 256,
//                a quarter of the trailing-matrix traffic of a 64-wide
//                right-looking update; 128x128 tiles, the tiles of one element
//                on one XCD (shared L2)
// then k_extract copies [S^K | g^K] out (column-major).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <climits>

#include "hdg_internal.h"

namespace hdg {
namespace {

// Matrix-core tile of 16x16 outputs with k = 4 per instruction, FP64 or FP32.
// Inputs: lane l holds A[l%16][l/16] and B[l/16][l%16]; output slot j of lane l
// holds row rowof(l, j), column l%16.
template <typename T> struct MF;
template <> struct MF<double> {
    typedef double acc_t __attribute__((ext_vector_type(4)));
    typedef double v2 __attribute__((ext_vector_type(2)));
    typedef double v16 __attribute__((ext_vector_type(2)));  // one 16-byte access
    static constexpr int V = 2;
    __device__ static acc_t mfma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static int rowof(int lane, int j) { return 4 * j + (lane >> 4); }
};
template <> struct MF<float> {
    typedef float acc_t __attribute__((ext_vector_type(4)));
    typedef float v2 __attribute__((ext_vector_type(2)));
    typedef float v16 __attribute__((ext_vector_type(4)));
    static constexpr int V = 4;
    __device__ static acc_t mfma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static int rowof(int lane, int j) { return 4 * (lane >> 4) + j; }
};

constexpr int kNB = 64;       // panel width
constexpr int kNBO = 128;     // pivot columns per trailing update
constexpr int kW = 8;         // register sub-panel width
constexpr int kHalf = 32;     // the panel is factored as two halves (sub-panels update only within a half)
constexpr int kPT = 512;      // panel kernel threads
constexpr int kRPC = 32;      // columns per k_rowperm workgroup
constexpr int kBC = 64;       // columns per k_blocku workgroup
constexpr int kCR = 128;      // trace rows per k_crows workgroup
static_assert(kW >= 8 && kPT >= 2 * 64, "panel scratch and permutation assumptions");
// A recorded permutation of w swaps (row base+jj <-> piv[jj]): [0] = number of
// displaced rows, [1 .. W] source row of each top row, then (dst, src) pairs.
constexpr int kPerm64 = 1 + kNB + 2 * kNB;
constexpr int kPerm128 = 1 + kNBO + 2 * kNBO;
// Workspace of one element and one 128-column block: values [6][64*64] (L^{-1}
// of panels 0, 1, then U^{-1} of panels 0, 1, then the off-diagonal blocks Lc
// and Uc of the 128-row inverses, see k_inv128), then ints: piv[128] | perm of
// panel 0 | perm of panel 1 | perm of the 128 block.  The FP64 path reuses one
// block's worth per element; the mixed path keeps every block (its solves
// replay them).
constexpr int kWsDbl = 6 * kNB * kNB;
constexpr int kWsLc = 4 * kNB * kNB, kWsUc = 5 * kNB * kNB;
constexpr int kWsPiv = 0, kWsPerm0 = kNBO, kWsPerm1 = kWsPerm0 + kPerm64, kWsPerm128 = kWsPerm1 + kPerm64;
constexpr int kWsInt = kWsPerm128 + kPerm128;

template <typename T> struct WS {
    T *d;        // element 0's values of the current block
    int *i;      // element 0's ints of the current block
    int64_t ds;  // per-element stride of d (values)
    int64_t is;  // per-element stride of i (ints)
};

struct ElemDims {
    int n, f, mrows, ncols;  // pivot columns, trace size, rows, columns
    int64_t ld;
};
// Systems factored here: mode 0 = element systems (n = 20 N_p, f = f_e, all
// n + f rows); mode 1 = Schwarz inversion systems [S_r | I] (n = f = f_r rounded up
// to a multiple of 4, n rows); mode 2 = FP32 interior rows [A | B R_qu] (n rows).
struct SysDesc {
    int mode;
    const int64_t *off;  // [n_elem+1] offsets (elements) of the systems
};
__device__ inline ElemDims elem_dims(const DevMesh &dm, const SysDesc &sd, int e) {
    ElemDims d;
    if (sd.mode != 1) {
        const int p = dm.elem_p[e];
        d.n = 20 * (p + 1) * (p + 1) * (p + 1);
        d.f = dm.toff[7 * e + 6];
    } else {
        // Schwarz system padded with decoupled unknowns to a multiple of 4
        d.n = asm_pad(dm.toff[7 * e + 6]);
        d.f = d.n;
    }
    d.mrows = (sd.mode == 0) ? d.n + d.f : d.n;
    d.ncols = d.n + d.f + 1;
    d.ld = e_ld(d.n, d.f);
    return d;
}

template <typename T> __device__ inline void argmax_combine(T &v, int &r, T v2, int r2) {
    const bool take = (v2 > v) | ((v2 == v) & (r2 < r));  // selects, no branches
    v = take ? v2 : v;
    r = take ? r2 : r;
}

// Lane exchange by a DPP pattern (a VALU operand modifier, no LDS round trip).
template <int CTRL> __device__ inline int dpp_int(int x) { return __builtin_amdgcn_update_dpp(x, x, CTRL, 0xF, 0xF, false); }
template <int CTRL> __device__ inline float dpp_val(float x) { return __int_as_float(dpp_int<CTRL>(__float_as_int(x))); }
template <int CTRL> __device__ inline double dpp_val(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = dpp_int<CTRL>((int)b), hi = dpp_int<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL, typename T> __device__ inline void argmax_dpp(T &v, int &r) {
    argmax_combine(v, r, dpp_val<CTRL>(v), dpp_int<CTRL>(r));
}
// Lane pairs (l, l ^ 16) or (l, l ^ 32) by the gfx950 row swaps: with both
// operands the same register, the two results hold, lane by lane, the lane's own
// value and its partner's (in some order), which is all a symmetric combine needs.
template <int W> __device__ inline void swap_pair(unsigned x, unsigned &a, unsigned &b) {
    const auto p = (W == 16) ? __builtin_amdgcn_permlane16_swap(x, x, false, false)
                             : __builtin_amdgcn_permlane32_swap(x, x, false, false);
    a = p[0];
    b = p[1];
}
template <int W> __device__ inline void argmax_swap(float &v, int &r) {
    unsigned va, vb, ra, rb;
    swap_pair<W>(__float_as_uint(v), va, vb);
    swap_pair<W>((unsigned)r, ra, rb);
    v = __uint_as_float(va);
    r = (int)ra;
    argmax_combine(v, r, __uint_as_float(vb), (int)rb);
}
template <int W> __device__ inline void argmax_swap(double &v, int &r) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    unsigned la, lb, ha, hb, ra, rb;
    swap_pair<W>((unsigned)b, la, lb);
    swap_pair<W>((unsigned)(b >> 32), ha, hb);
    swap_pair<W>((unsigned)r, ra, rb);
    v = __longlong_as_double((long long)(((unsigned long long)ha << 32) | la));
    r = (int)ra;
    argmax_combine(v, r, __longlong_as_double((long long)(((unsigned long long)hb << 32) | lb)), (int)rb);
}
// Wave-wide argmax (largest value, smallest row on ties), the result in every
// lane.  The combine is associative and commutative, so the order of the steps
// does not change the result: quad permutations [1,0,3,2] and [2,3,0,1] and
// rotations by 4 and 8 inside each 16-lane row, then the row swaps across 16 and
// 32 lanes.  No step goes through LDS.
template <typename T> __device__ inline void wave_argmax(T &v, int &r) {
    argmax_dpp<0xB1>(v, r);   // quad_perm [1,0,3,2]
    argmax_dpp<0x4E>(v, r);   // quad_perm [2,3,0,1]
    argmax_dpp<0x124>(v, r);  // row_ror 4
    argmax_dpp<0x128>(v, r);  // row_ror 8
    argmax_swap<16>(v, r);
    argmax_swap<32>(v, r);
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

// XCD-aware work mapping: consecutive workgroups go round-robin over the 8 XCDs;
// XCD x takes elements x, x+8, x+16, ... with all their tiles, so an element's
// tiles share one L2 and every XCD gets an equal share of the element sizes
// however the elements are ordered.  False past the last element.
__device__ inline bool xcd_item(int ne, int tiles, int &el, int &t) {
    const int xcd = blockIdx.x % 8, idx = blockIdx.x / 8;
    el = 8 * (idx / tiles) + xcd;
    t = idx % tiles;
    return el < ne;
}
inline int xcd_grid(int ne, int tiles) { return 8 * ((ne + 7) / 8) * tiles; }

// ------------------------------------------------------------------ panel
// Factor the panel columns [k0, k0+nb) over the pivot rows [k0, n) (the trace
// rows n.. get their multipliers from k_crows).  Rows are distributed over the
// threads (row cb + tid + kPT i), kW columns at a time held in registers.  The
// panel is two halves factored by two launches (part 1, part 2): sub-panels
// update the columns of their own half only; part 1 ends with the first half's
// U12 rows, and the second half receives the whole first half's update from
// k_half (matrix cores, many workgroups) between the launches, which reads and
// writes the panel's right part far fewer times.
template <int R, int TAG, typename T>
__global__ void __launch_bounds__(kPT, sizeof(T) == 4 ? 4 : 2) k_panel(DevMesh dm, SysDesc sd, int e0, int k0, int slot, int kbase, int part,
                                               T *__restrict__ Ebase, WS<T> ws, int *__restrict__ info) {
    constexpr int kVN = 16 / sizeof(T);  // values per 16-byte access
    typedef T vq __attribute__((ext_vector_type(kVN)));
    const int e = e0 + blockIdx.x;
    const ElemDims dd = elem_dims(dm, sd, e);
    if (k0 >= dd.n) return;
    const int nb = min(kNB, dd.n - k0);
    const int n = dd.n;
    T *E = Ebase + (sd.off[e] - sd.off[e0]);
    const int64_t ld = dd.ld;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    __shared__ T s_val[kPT / 64];
    __shared__ int s_row[kPT / 64];
    __shared__ T s_prow[kW], s_krow[kW];
    __shared__ int s_piv[kNBO];
    __shared__ int s_top[kNB], s_disp[2 * kNB], s_nd;
    __shared__ T s_L[kW][kW];
    __shared__ T s_U[kW][kNB];
    __shared__ int s_piv2[kNBO], s_wcnt[2];
    __shared__ T s_T[kNB][kNB + 1], s_I[kNB][kNB + 1];
    int info_k = 0;
    // part 1: the first half (ending with its U12 rows), part 2: the second
    // half and the records; a panel of at most kHalf columns is done by part 1
    const bool split = nb > kHalf;
    if (part == 2 && !split) return;
    int *wi = ws.i + (int64_t)blockIdx.x * ws.is;
    const int j_begin = (part == 2) ? kHalf : 0, j_end = (part == 1 && split) ? kHalf : nb;
    if (part == 2) {
        for (int t = tid; t < kHalf; t += kPT) s_piv[t] = wi[kWsPiv + slot * kNB + t];
        __syncthreads();
    }

    for (int j0 = j_begin; j0 < j_end; j0 += kW) {
        const int w = min(kW, nb - j0), cb = k0 + j0;
        T a[R][kW];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int r = cb + tid + kPT * i;
            const T *src = E + (int64_t)min(r, n - 1) * ld + cb;
            if (w == kW) {
                // 16-byte loads (cb is a multiple of kW, ld of 8)
#pragma unroll
                for (int c = 0; c < kW; c += kVN) {
                    const vq v = *(const vq *)(src + c);
#pragma unroll
                    for (int u = 0; u < kVN; ++u) a[i][c + u] = (r < n) ? v[u] : T(0);
                }
            } else {
#pragma unroll
                for (int c = 0; c < kW; ++c) a[i][c] = (r < n && c < w) ? src[c] : T(0);
            }
        }
#pragma unroll
        for (int jj = 0; jj < kW; ++jj) {
            if (jj < w) {  // uniform; keeps jj a compile-time register index
            const int k = cb + jj;
            // pivot: largest |a| over rows k..n-1 (smallest row index on ties); NaN wins
            T best = T(-1);
            int brow = INT_MAX;
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int r = cb + tid + kPT * i;
                if (r >= k && r < n) {
                    T v = fabs(a[i][jj]);
                    if (!(v == v)) v = T(INFINITY);
                    argmax_combine(best, brow, v, r);
                }
            }
            wave_argmax(best, brow);
            if (lane == 0) { s_val[wave] = best; s_row[wave] = brow; }
            __syncthreads();
            T bv = s_val[0];
            int pr = s_row[0];
#pragma unroll
            for (int t = 1; t < kPT / 64; ++t) argmax_combine(bv, pr, s_val[t], s_row[t]);
            const bool bad = !(bv > T(0)) || !(bv < T(INFINITY)) || pr == INT_MAX;
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
            const T pinv = bad ? T(0) : T(1) / s_prow[jj];
            T prow[kW];
#pragma unroll
            for (int c = jj + 1; c < kW; ++c) prow[c] = s_prow[c];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int r = cb + tid + kPT * i;
                if (r > k && r < n) {
                    const T l = a[i][jj] * pinv;
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
            T *dst = E + (int64_t)r * ld + cb;
            if (r < n && w == kW) {
#pragma unroll
                for (int c = 0; c < kW; c += kVN) {
                    vq v;
#pragma unroll
                    for (int u = 0; u < kVN; ++u) v[u] = a[i][c + u];
                    *(vq *)(dst + c) = v;
                }
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
            T vals[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int t = tid + q * kPT;
                vals[q] = T(0);
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
        // sub-panels of the first half update only the first half's columns; the
        // second half receives the first half's update in one pass below
        const int nrloc = (j0 + w <= kHalf && split) ? kHalf - j0 - w : nright;
        if (nrloc > 0) {
            // U of the sub-panel rows in the right columns: unit lower solve
            for (int cidx = tid; cidx < nrloc; cidx += kPT) {
                const int col = cb + w + cidx;
                T x[kW];
#pragma unroll
                for (int r = 0; r < kW; ++r) x[r] = (r < w) ? E[(int64_t)(cb + r) * ld + col] : T(0);
#pragma unroll
                for (int r = 0; r < kW; ++r)
#pragma unroll
                    for (int rr = 0; rr < r; ++rr) x[r] -= s_L[r][rr] * x[rr];
#pragma unroll
                for (int r = 0; r < kW; ++r) {
                    if (r < w) E[(int64_t)(cb + r) * ld + col] = x[r];
                    s_U[r][cidx] = (r < w) ? x[r] : T(0);
                }
            }
            __syncthreads();
            // pivot rows below the sub-panel: E[r][right] -= L[r][0:w] U[0:w][right].
            // Each thread walks its own rows, so every access of a wave touches 64
            // rows: 16-byte accesses halve (FP64) or quarter (FP32) their number.
            // Aligned: nrloc > 0 only for w = kW, cb is a multiple of kW, ld of 8,
            // and nrloc of 4, so no 16-byte group straddles the end of the range.
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int r = cb + tid + kPT * i;
                if (r < cb + w || r >= n) continue;
                T *row = E + (int64_t)r * ld + cb + w;
                for (int c8 = 0; c8 < nrloc; c8 += 8) {
                    T v[8];
#pragma unroll
                    for (int h = 0; h < 8; h += kVN) {
                        vq x = (vq)T(0);
                        if (c8 + h < nrloc) x = *(const vq *)(row + c8 + h);
#pragma unroll
                        for (int u = 0; u < kVN; ++u) v[h + u] = x[u];
                    }
#pragma unroll
                    for (int jj = 0; jj < kW; ++jj)
#pragma unroll
                        for (int q = 0; q < 8; ++q) v[q] -= a[i][jj] * s_U[jj][(c8 + q) & (kNB - 1)];
#pragma unroll
                    for (int h = 0; h < 8; h += kVN) {
                        if (c8 + h < nrloc) {
                            vq x;
#pragma unroll
                            for (int u = 0; u < kVN; ++u) x[u] = v[h + u];
                            *(vq *)(row + c8 + h) = x;
                        }
                    }
                }
            }
            __syncthreads();
        }
        if (split && j0 + w == kHalf) {
            // second half: U12 = L11^{-1} A12 on the top kHalf rows (one thread per
            // column); A22 -= L21 U12 for the rows below is k_half's, between the
            // two launches
            const int nb2 = nb - kHalf;
            for (int t = tid; t < kHalf * kHalf; t += kPT) {
                const int r = t / kHalf, c = t % kHalf;
                s_T[r][c] = E[(int64_t)(k0 + r) * ld + k0 + c];
                s_I[r][c] = (c < nb2) ? E[(int64_t)(k0 + r) * ld + k0 + kHalf + c] : T(0);
            }
            __syncthreads();
            if (tid < nb2) {
                for (int r = 1; r < kHalf; ++r) {
                    T x = s_I[r][tid];
                    for (int rr = 0; rr < r; ++rr) x -= s_T[r][rr] * s_I[rr][tid];
                    s_I[r][tid] = x;
                }
            }
            __syncthreads();
            for (int t = tid; t < kHalf * nb2; t += kPT) {
                const int r = t / nb2, c = t % nb2;
                E[(int64_t)(k0 + r) * ld + k0 + kHalf + c] = s_I[r][c];
            }
        }
    }
    if (part == 1 && split) {
        // first half done: its pivots go to the workspace for the second launch
        for (int t = tid; t < kHalf; t += kPT) wi[kWsPiv + slot * kNB + t] = s_piv[t];
        if (tid == 0 && info_k && info[e] == 0) info[e] = info_k;
        return;
    }
    // record pivots, the panel's net permutation, L11^{-1} and U11^{-1}
    T *wd = ws.d + (int64_t)blockIdx.x * ws.ds;
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
        s_T[r][c] = (r < nb && c < nb) ? E[(int64_t)(k0 + r) * ld + k0 + c] : T(0);
        s_I[r][c] = T(0);
    }
    __syncthreads();
    // Both inverses by 8 x 8 block substitution over the whole block: first the
    // diagonal blocks (one thread per column), then one block row at a time,
    // P = (off-diagonal part of the row) x (finished rows of the inverse) and
    // X_row = -X_diag P.  Rows and columns >= nb act as identity and are
    // returned as zero.
    T (*s_P)[kNB] = s_U;  // [8][64] partial products
    if (tid < kNB) {
        // diagonal block of L11^{-1}: forward substitution, unit diagonal
        const int j = tid, bi = j & ~7, jl = j & 7;
        T x[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            T v = (r == jl) ? T(1) : T(0);
#pragma unroll
            for (int c = 0; c < r; ++c) v -= s_T[bi + r][bi + c] * x[c];
            x[r] = (r >= jl) ? v : T(0);
            s_I[bi + r][j] = x[r];
        }
    }
    __syncthreads();
    for (int bI = 8; bI < kNB; bI += 8) {
        const int i = tid & 7, j = tid >> 3;  // j < bI: columns left of the block row
        if (j < bI) {
            T v = T(0);
            for (int k = j & ~7; k < bI; ++k) v += s_T[bI + i][k] * s_I[k][j];
            s_P[i][j] = v;
        }
        __syncthreads();
        if (j < bI) {
            T v = T(0);
#pragma unroll
            for (int c = 0; c < 8; ++c) v -= s_I[bI + i][bI + c] * s_P[c][j];
            s_I[bI + i][j] = v;
        }
        __syncthreads();
    }
    T *li = wd + slot * kNB * kNB;
    for (int t = tid; t < kNB * kNB; t += kPT) {
        const int r = t / kNB, c = t % kNB;
        li[t] = (r < nb && c < nb) ? s_I[r][c] : T(0);
    }
    __syncthreads();
    for (int t = tid; t < kNB * kNB; t += kPT) s_I[t / kNB][t % kNB] = T(0);
    __syncthreads();
    if (tid < kNB) {
        // diagonal block of U11^{-1}: back substitution
        const int j = tid, bi = j & ~7, jl = j & 7;
        T x[8];
#pragma unroll
        for (int r = 7; r >= 0; --r) {
            T v = (r == jl) ? T(1) : T(0);
#pragma unroll
            for (int c = r + 1; c < 8; ++c) v -= s_T[bi + r][bi + c] * x[c];
            const T d = (bi + r < nb) ? s_T[bi + r][bi + r] : T(1);
            x[r] = (r <= jl) ? v / d : T(0);
            s_I[bi + r][j] = x[r];
        }
    }
    __syncthreads();
    for (int bI = kNB - 16; bI >= 0; bI -= 8) {
        const int i = tid & 7, j = bI + 8 + (tid >> 3);  // columns right of the block row
        if (j < kNB) {
            T v = T(0);
            for (int k = bI + 8; k <= (j | 7); ++k) v += s_T[bI + i][k] * s_I[k][j];
            s_P[i][j] = v;
        }
        __syncthreads();
        if (j < kNB) {
            T v = T(0);
#pragma unroll
            for (int c = 0; c < 8; ++c) v -= s_I[bI + i][bI + c] * s_P[c][j];
            s_I[bI + i][j] = v;
        }
        __syncthreads();
    }
    T *ui = wd + (2 + slot) * kNB * kNB;
    for (int t = tid; t < kNB * kNB; t += kPT) {
        const int r = t / kNB, c = t % kNB;
        ui[t] = (r < nb && c < nb) ? s_I[r][c] : T(0);
    }
    if (tid == 0 && info_k && info[e] == 0) info[e] = info_k;
}

// acc (rows 16 wave .. +15, C columns) = Ls (64x64) * X (64 x C), both in LDS.
template <typename T, int C>
__device__ inline void mfma_64xc(const T (*Ls)[kNB + 1], const T (*X)[C + 1], typename MF<T>::acc_t acc[C / 16],
                                 int lane, int wave) {
#pragma unroll
    for (int j = 0; j < C / 16; ++j) acc[j] = (typename MF<T>::acc_t){T(0), T(0), T(0), T(0)};
#pragma unroll 4
    for (int kk = 0; kk < kNB; kk += 4) {
        const T a = Ls[16 * wave + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
        for (int j = 0; j < C / 16; ++j) {
            const T b = X[kk + (lane >> 4)][16 * j + (lane & 15)];
            acc[j] = MF<T>::mfma(a, b, acc[j]);
        }
    }
}

template <typename T>
__device__ inline void mfma_64x64(const T (*Ls)[kNB + 1], const T (*X)[65], typename MF<T>::acc_t acc[4], int lane,
                                  int wave) {
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = (typename MF<T>::acc_t){T(0), T(0), T(0), T(0)};
#pragma unroll 4
    for (int kk = 0; kk < kNB; kk += 4) {
        const T a = Ls[16 * wave + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const T b = X[kk + (lane >> 4)][16 * j + (lane & 15)];
            acc[j] = MF<T>::mfma(a, b, acc[j]);
        }
    }
}

// acc[j] += A[r][k] X[xoff + k][16 j + cl] over k in [k_lo, k_hi) (multiples of
// 16) for the lane's row r: arow[k] = A[r][k + kq], fragments in matrix-core
// order (kq = lane / 16, cl = lane % 16), A from the cache, X from LDS.  Four
// A loads are issued per 16-wide chunk before its products.
template <typename T, int NJ, int LDX>
__device__ inline void mfma_rowblock(const T *arow, const T (*X)[LDX], int xoff, int k_lo, int k_hi, int kq, int cl,
                                     typename MF<T>::acc_t *acc) {
    for (int kb = k_lo; kb < k_hi; kb += 16) {
        T a[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] = arow[kb + 4 * q];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int j = 0; j < NJ; ++j) acc[j] = MF<T>::mfma(a[q], X[xoff + kb + 4 * q + kq][16 * j + cl], acc[j]);
    }
}

// A22 -= L21 U12 between the two halves of the panel at kp: pivot rows
// kp+32 .. n-1, columns kp+32 .. kp+nb-1, K = 32.  64 rows per workgroup (16
// per wave), U12 (zero beyond nb) in LDS, L21 fragments from the cache.
template <int TAG, typename T>
__global__ void __launch_bounds__(256) k_half(DevMesh dm, SysDesc sd, int e0, int kp, T *__restrict__ Ebase) {
    typedef typename MF<T>::acc_t acc_t;
    const int e = e0 + blockIdx.y;
    const ElemDims dd = elem_dims(dm, sd, e);
    if (kp >= dd.n) return;
    const int nb = min(kNB, dd.n - kp);
    if (nb <= kHalf) return;
    const int nb2 = nb - kHalf;
    const int r0 = kp + kHalf + blockIdx.x * 64;
    if (r0 >= dd.n) return;  // uniform per block
    T *E = Ebase + (sd.off[e] - sd.off[e0]);
    const int64_t ld = dd.ld;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int kq = lane >> 4, cl = lane & 15;
    __shared__ T sU[kHalf][kHalf + 1];
    for (int t = tid; t < kHalf * kHalf; t += 256) {
        const int r = t / kHalf, c = t % kHalf;
        sU[r][c] = (c < nb2) ? E[(int64_t)(kp + r) * ld + kp + kHalf + c] : T(0);
    }
    __syncthreads();
    const int rb = r0 + 16 * wave;
    if (rb >= dd.n) return;  // uniform per wave; no barrier follows
    acc_t acc[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[j] = (acc_t){T(0), T(0), T(0), T(0)};
    const int ra = min(rb + cl, dd.n - 1);
    mfma_rowblock<T, 2>(E + (int64_t)ra * ld + kp + kq, sU, 0, 0, kHalf, kq, cl, acc);
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = rb + MF<T>::rowof(lane, q), c = 16 * j + cl;
            if (r < dd.n && c < nb2) {
                T *dst = E + (int64_t)r * ld + kp + kHalf + c;
                *dst = *dst - acc[j][q];
            }
        }
}

// Multipliers of the trace rows n..n+f-1 in the panel columns [kp, kp+nb):
// L_C = C_panel U11^{-1} (matrix cores), in place, one workgroup per 128 trace
// rows: U11^{-1} in LDS, the C rows read from the cache as matrix-core operands,
// each wave on its own 32 rows.
template <int TAG, typename T>
__global__ void __launch_bounds__(256) k_crows(DevMesh dm, SysDesc sd, int e0, int kp, int slot,
                                               T *__restrict__ Ebase, WS<T> ws) {
    typedef typename MF<T>::acc_t acc_t;
    const int e = e0 + blockIdx.y;
    const ElemDims dd = elem_dims(dm, sd, e);
    if (kp >= dd.n) return;
    const int nb = min(kNB, dd.n - kp);
    const int r0 = dd.n + blockIdx.x * kCR;
    if (r0 >= dd.mrows) return;  // uniform per block
    T *E = Ebase + (sd.off[e] - sd.off[e0]);
    const int64_t ld = dd.ld;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int kq = lane >> 4, cl = lane & 15;
    __shared__ T sU[kNB][kNB + 1];
    const T *ui = ws.d + (int64_t)blockIdx.y * ws.ds + (2 + slot) * kNB * kNB;
    for (int t = tid; t < kNB * kNB; t += 256) sU[t >> 6][t & 63] = ui[t];
    __syncthreads();
    // K = nb rounded up to 16: U11^{-1} is zero beyond nb, and the C entries there
    // are finite (the next panel's columns, or the row padding)
    const int kend = (nb + 15) & ~15;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int rb = r0 + 32 * wave + 16 * h;
        if (rb >= dd.mrows) break;  // uniform per wave; no barrier follows
        acc_t acc[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = (acc_t){T(0), T(0), T(0), T(0)};
        const int ra = min(rb + cl, dd.mrows - 1);
        mfma_rowblock<T, 4>(E + (int64_t)ra * ld + kp + kq, sU, 0, 0, kend, kq, cl, acc);
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = rb + MF<T>::rowof(lane, q), c = 16 * j + cl;
                if (r < dd.mrows && c < nb) E[(int64_t)r * ld + kp + c] = acc[j][q];
            }
    }
}

// ------------------------------------------------------- row permutation
// MODE 0: rows base..base+63 <- permuted (panel 0), U = L^{-1} X, on
//         columns [k0 + K_e, k0 + min(CW, n_e - k0))  (CW = 0: to the end)
// MODE 1: permutation of panel 1 only, on the columns of panel 0 (its L)
// One workgroup per (32-column tile, element).  (The 128-row block of the
// trailing columns is k_blocku's.)
template <int MODE, int TAG, typename T>
__global__ void __launch_bounds__(256) k_rowperm(DevMesh dm, SysDesc sd, int e0, int k0, int CW,
                                                 T *__restrict__ Ebase, WS<T> ws) {
    typedef typename MF<T>::acc_t acc_t;
    const int e = e0 + blockIdx.y;
    const ElemDims dd = elem_dims(dm, sd, e);
    if (k0 >= dd.n) return;
    const int rem = dd.n - k0;
    int c_begin, c_end, base, nrows, permoff;
    if (MODE == 0) {
        const int K = min(kNB, rem);
        c_begin = k0 + K;
        c_end = CW > 0 ? k0 + min(CW, rem) : dd.ncols;
        base = k0; nrows = K; permoff = kWsPerm0;
    } else {
        if (rem <= kNB) return;
        c_begin = k0;
        c_end = k0 + kNB;
        base = k0 + kNB; nrows = min(kNB, rem - kNB); permoff = kWsPerm1;
    }
    const int c0 = c_begin + blockIdx.x * kRPC;
    if (c0 >= c_end) return;  // uniform per block
    T *E = Ebase + (sd.off[e] - sd.off[e0]);
    const int64_t ld = dd.ld;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    __shared__ T sX[kNB][kRPC + 1];
    __shared__ T sM[kNB][kNB + 1];
    __shared__ int sperm[kPerm64];
    const int *wi = ws.i + (int64_t)blockIdx.y * ws.is;
    constexpr int W = kNB;
    const int permlen = 1 + W + 2 * W;
    for (int t = tid; t < permlen; t += 256) sperm[t] = wi[permoff + t];
    __syncthreads();
    // gather the permuted top rows, then move the displaced rows
    for (int t = tid; t < nrows * kRPC; t += 256) {
        const int r = t / kRPC, c = t % kRPC;
        sX[r][c] = (c0 + c < c_end) ? E[(int64_t)sperm[1 + r] * ld + c0 + c] : T(0);
    }
    for (int t = tid; t < (kNB - nrows) * kRPC; t += 256) sX[nrows + t / kRPC][t % kRPC] = T(0);
    // a top row's source may be a displaced row: its old content must be read
    // before the displaced copies overwrite it
    __syncthreads();
    // displaced rows take original top rows, which are rewritten only after the
    // next barrier
    const int nd = sperm[0];
    for (int t = tid; t < nd * kRPC; t += 256) {
        const int d = t / kRPC, c = t % kRPC;
        if (c0 + c < c_end) {
            const int dst = sperm[1 + W + 2 * d], src = sperm[1 + W + 2 * d + 1];
            E[(int64_t)dst * ld + c0 + c] = E[(int64_t)src * ld + c0 + c];
        }
    }
    if (MODE == 1) __syncthreads();
    if (MODE == 0) {
        const T *la = ws.d + (int64_t)blockIdx.y * ws.ds;
        acc_t acc[kRPC / 16];
        // U_a = La^{-1} X_a
        for (int t = tid; t < kNB * kNB; t += 256) sM[t >> 6][t & 63] = la[t];
        __syncthreads();
        mfma_64xc<T, kRPC>(sM, sX, acc, lane, wave);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kRPC / 16; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) sX[16 * wave + MF<T>::rowof(lane, q)][16 * j + (lane & 15)] = acc[j][q];
        __syncthreads();
    }
    for (int t = tid; t < nrows * kRPC; t += 256) {
        const int r = t / kRPC, c = t % kRPC;
        if (c0 + c < c_end) E[(int64_t)(base + r) * ld + c0 + c] = sX[r][c];
    }
}

// ------------------------------------------------ 128-row block inverses
// The unit lower and the upper triangle of a 128-column block (panels a and b)
// have the inverses [[La^{-1}, 0], [Lc, Lb^{-1}]], Lc = -Lb^{-1} L_ba La^{-1},
// and [[Ua^{-1}, Uc], [0, Ub^{-1}]], Uc = -Ua^{-1} U_ab Ub^{-1}.  k_inv128 forms
// Lc and Uc once per element, after panel b's swaps have reached L_ba (rows
// base+64.., columns base..base+63 of E); U_ab (rows base.., columns base+64..)
// is final once panel a's U rows are formed.  Both go to the block's workspace.
template <int TAG, typename T>
__global__ void __launch_bounds__(256) k_inv128(DevMesh dm, SysDesc sd, int e0, int k0, const T *__restrict__ Ebase,
                                                WS<T> ws) {
    // products in FP64 whatever T is, rounded to T once (the FP32 path's
    // explicit blocks then carry one rounding, not three)
    typedef typename MF<double>::acc_t acc_t;
    const int e = e0 + blockIdx.x;
    const ElemDims dd = elem_dims(dm, sd, e);
    if (k0 >= dd.n || dd.n - k0 <= kNB) return;
    const int nb1 = min(kNB, dd.n - k0 - kNB);
    const T *E = Ebase + (sd.off[e] - sd.off[e0]);
    const int64_t ld = dd.ld;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    __shared__ double sL[kNB][kNB + 1], sR[kNB][kNB + 1];
    T *wd = ws.d + (int64_t)blockIdx.x * ws.ds;
    acc_t acc[4];
    // -(F G H) for 64 x 64 blocks: F from the workspace slot f_slot, G from E at
    // (g_row, g_col) with rows (or columns) >= nb1 zero, H from slot h_slot;
    // the result goes to slot out.
    auto triple = [&](int f_slot, int g_row, int g_col, bool g_rows, int h_slot, int out) {
        for (int t = tid; t < kNB * kNB; t += 256) {
            const int r = t >> 6, c = t & 63;
            sL[r][c] = ((g_rows ? r : c) < nb1) ? (double)E[(int64_t)(g_row + r) * ld + g_col + c] : 0.0;
            sR[r][c] = (double)wd[h_slot + t];
        }
        __syncthreads();
        mfma_64x64<double>(sL, sR, acc, lane, wave);  // G H
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) sR[16 * wave + MF<double>::rowof(lane, q)][16 * j + (lane & 15)] = acc[j][q];
        for (int t = tid; t < kNB * kNB; t += 256) sL[t >> 6][t & 63] = (double)wd[f_slot + t];
        __syncthreads();
        mfma_64x64<double>(sL, sR, acc, lane, wave);  // F (G H)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                wd[out + (16 * wave + MF<double>::rowof(lane, q)) * kNB + 16 * j + (lane & 15)] = (T)(-acc[j][q]);
        __syncthreads();
    };
    triple(kNB * kNB, k0 + kNB, k0, true, 0, kWsLc);                     // Lc = -Lb^{-1} L_ba La^{-1}
    triple(2 * kNB * kNB, k0, k0 + kNB, false, 3 * kNB * kNB, kWsUc);    // Uc = -Ua^{-1} U_ab Ub^{-1}
}

// One kBC-column tile of a block of nrows = min(128, n - k0) pivot columns
// applied to other columns: X = P A12 (the block's net row permutation: permuted
// top rows gathered into LDS, displaced rows moved), then U12 = L11^{-1} X in a
// single product with the recorded inverse.  The zero blocks of the triangle
// are skipped; wave w takes the 16-row blocks w and 7 - w, whose inner lengths
// 16 (w + 1) and 16 (8 - w) give every wave the same work.  L11^{-1} is read
// from the cache in matrix-core operand order, X from LDS.  Columns: from
// k0 + max(nrows, min(CB, n - k0)) to k0 + min(CW, n - k0) (CW > 0) or to the
// last column; rhs = 1: the right-hand columns n.. only (replays the block's
// forward substitution).
//   MODE 0  as above.
//   MODE 1  the second block B of a pair (A, B = rows k0-128..k0-1, k0..): the
//           columns still lack A's update, which is applied to the gathered
//           rows only, X -= L_A[top rows] U12_A (A's L after B's swaps, A's U
//           rows of the tile), before the solve.  The displaced rows keep A's
//           update pending with their L_A rows.
//   MODE 2  B's swaps on the columns of A's L (k0-128 .. k0-1), no solve.
// One workgroup per (tile, element); an element's tiles share an XCD.
template <int MODE, int TAG, typename T>
__global__ void __launch_bounds__(256) k_blocku(DevMesh dm, SysDesc sd, int e0, int ne, int k0, int rhs, int CB,
                                                int CW, int tiles, T *__restrict__ Ebase, WS<T> ws) {
    typedef typename MF<T>::acc_t acc_t;
    int el, tl;
    if (!xcd_item(ne, tiles, el, tl)) return;
    const int e = e0 + el;
    const ElemDims dd = elem_dims(dm, sd, e);
    if (k0 >= dd.n) return;
    const int rem = dd.n - k0, nrows = min(kNBO, rem);
    int c_begin, c_end;
    if (MODE == 2) {
        c_begin = k0 - kNBO;
        c_end = k0;
    } else if (rhs) {
        c_begin = dd.n;
        c_end = dd.ncols;
    } else {
        c_begin = k0 + max(nrows, min(CB, rem));
        c_end = CW > 0 ? k0 + min(CW, rem) : dd.ncols;
    }
    const int c0 = c_begin + tl * kBC;
    if (c0 >= c_end) return;  // uniform per block
    T *E = Ebase + (sd.off[e] - sd.off[e0]);
    const int64_t ld = dd.ld;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    __shared__ T sX[kNBO][kBC + 1];
    __shared__ int sperm[kPerm128];
    const int *wi = ws.i + (int64_t)el * ws.is;
    const T *wd = ws.d + (int64_t)el * ws.ds;
    const bool two = nrows > kNB;
    const int W = two ? kNBO : kNB;
    const int permoff = two ? kWsPerm128 : kWsPerm0;
    for (int t = tid; t < 1 + 3 * W; t += 256) sperm[t] = wi[permoff + t];
    __syncthreads();
    // gather the permuted top rows (rows >= nrows are zero): all loads in flight
    // from clamped in-range addresses, the out-of-range entries zeroed at the store
    {
        constexpr int kG = kNBO * kBC / 256;
        T g[kG];
#pragma unroll
        for (int q = 0; q < kG; ++q) {
            const int t = tid + 256 * q;
            const int r = t / kBC, c = t % kBC;
            g[q] = E[(int64_t)sperm[1 + min(r, nrows - 1)] * ld + min(c0 + c, c_end - 1)];
        }
#pragma unroll
        for (int q = 0; q < kG; ++q) {
            const int t = tid + 256 * q;
            const int r = t / kBC, c = t % kBC;
            sX[r][c] = (r < nrows && c0 + c < c_end) ? g[q] : T(0);
        }
    }
    // a top row's source may be a displaced row: its old content must be read
    // before the displaced copies overwrite it
    __syncthreads();
    // displaced rows take original top rows, which are rewritten only after the
    // next barrier
    const int nd = sperm[0];
    for (int t0 = tid; t0 < nd * kBC; t0 += 4 * 256) {
        T v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {  // clamped in-range reads, all in flight
            const int t = t0 + 256 * q, d = min(t / kBC, nd - 1), c = t % kBC;
            v[q] = E[(int64_t)sperm[1 + W + 2 * d + 1] * ld + min(c0 + c, c_end - 1)];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int t = t0 + 256 * q, d = t / kBC, c = t % kBC;
            if (t < nd * kBC && c0 + c < c_end) E[(int64_t)sperm[1 + W + 2 * d] * ld + c0 + c] = v[q];
        }
    }
    const int kq = lane >> 4, cl = lane & 15;
    if (MODE == 1) {
        // X -= L_A[k0 + r][k0-128 ..] U12_A, rows of blocks w and 7 - w
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int rb = h == 0 ? wave : 7 - wave;
            if (16 * rb >= nrows) continue;  // uniform per wave
            acc_t a[kBC / 16];
#pragma unroll
            for (int j = 0; j < kBC / 16; ++j) a[j] = (acc_t){T(0), T(0), T(0), T(0)};
            // both operands from the cache: L_A rows (lane's row) and U12_A (lane's
            // column; columns past the last one are read at the last column and
            // zeroed before use).  The next 16-wide step's operands are loaded
            // while the current step's products run.
            const int r = min(k0 + 16 * rb + cl, dd.n - 1);
            const T *arow = E + (int64_t)r * ld + k0 - kNBO + kq;
            const T *bcol[kBC / 16];
            bool cok[kBC / 16];
#pragma unroll
            for (int j = 0; j < kBC / 16; ++j) {
                const int col = c0 + 16 * j + cl;
                cok[j] = col < c_end;
                bcol[j] = E + (int64_t)(k0 - kNBO + kq) * ld + min(col, c_end - 1);
            }
            T av[2][4], bv[2][4][kBC / 16];
            auto load_step = [&](int kb, T (&ra)[4], T (&rb_)[4][kBC / 16]) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    ra[q] = arow[kb + 4 * q];
#pragma unroll
                    for (int j = 0; j < kBC / 16; ++j) rb_[q][j] = bcol[j][(int64_t)(kb + 4 * q) * ld];
                }
            };
            load_step(0, av[0], bv[0]);
#pragma unroll
            for (int s8 = 0; s8 < kNBO / 16; ++s8) {
                const int cur = s8 & 1;
                if (s8 + 1 < kNBO / 16) load_step(16 * (s8 + 1), av[cur ^ 1], bv[cur ^ 1]);
                __builtin_amdgcn_sched_barrier(0);  // keep the next step's loads ahead of these products
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int j = 0; j < kBC / 16; ++j)
                        a[j] = MF<T>::mfma(av[cur][q], cok[j] ? bv[cur][q][j] : T(0), a[j]);
            }
#pragma unroll
            for (int j = 0; j < kBC / 16; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int rr = 16 * rb + MF<T>::rowof(lane, q);
                    if (rr < nrows) sX[rr][16 * j + cl] -= a[j][q];
                }
        }
    }
    if (MODE == 2) {
        __syncthreads();
        for (int t = tid; t < nrows * kBC; t += 256) {
            const int r = t / kBC, c = t % kBC;
            if (c0 + c < c_end) E[(int64_t)(k0 + r) * ld + c0 + c] = sX[r][c];
        }
        return;
    }
    if (MODE == 1) __syncthreads();
    // U12 = L11^{-1} X
    acc_t acc[2][kBC / 16];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int rb = h == 0 ? wave : 7 - wave;
#pragma unroll
        for (int j = 0; j < kBC / 16; ++j) acc[h][j] = (acc_t){T(0), T(0), T(0), T(0)};
        if (16 * rb >= nrows) continue;  // uniform per wave
        const int r = 16 * rb + cl;
        if (rb < 4) {
            mfma_rowblock<T, kBC / 16>(wd + r * kNB + kq, sX, 0, 0, 16 * (rb + 1), kq, cl, acc[h]);  // La^{-1}
        } else {
            mfma_rowblock<T, kBC / 16>(wd + kWsLc + (r - kNB) * kNB + kq, sX, 0, 0, kNB, kq, cl, acc[h]);  // Lc
            mfma_rowblock<T, kBC / 16>(wd + kNB * kNB + (r - kNB) * kNB + kq, sX, kNB, 0, 16 * (rb - 3), kq, cl,
                                       acc[h]);  // Lb^{-1}
        }
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int rb = h == 0 ? wave : 7 - wave;
#pragma unroll
        for (int j = 0; j < kBC / 16; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = 16 * rb + MF<T>::rowof(lane, q), c = c0 + 16 * j + cl;
                if (r < nrows && c < c_end) E[(int64_t)(k0 + r) * ld + c] = acc[h][j][q];
            }
    }
}

// --------------------------------------------------------- trailing update
// C -= A B within one system, K = min(KW, n_e - k0) and A = E[rows, k0 .. k0+K),
// B = E[k0 .. k0+K, cols]:
//   kRangeLU:  rows [k0+K, mrows), columns from k0 + max(K, min(CB, n_e-k0)) to
//              k0+min(CW, n_e-k0) (CW > 0) or to ncols  (the LU's trailing update)
//   kRangeFwd: rows [k0+K, n), columns [n, ncols)  (forward substitution of the
//              right-hand columns)
// TM x 128 tile per workgroup (TM = 128 or 256), K in chunks of 16 (FP64) or
// 32 (FP32) values double-buffered through LDS, matrix cores; C is read before
// the K loop.
constexpr int kRangeLU = 0, kRangeFwd = 1;
constexpr int kFold = 128;  // FP32 products are folded into C every kFold values of K
constexpr int kTM = 128, kTN = 128;
template <typename T> struct UpdCfg {
    static constexpr int V = MF<T>::V;
    static constexpr int KC = 8 * V;      // k per LDS chunk
    static constexpr int SA = KC + V;     // LDS row stride of the A chunk (rows x k)
    static constexpr int SB = kTN + 16;   // LDS row stride of the B chunk (k x columns)
    static constexpr int LPK = kTN / V;   // lanes per k-row of the B chunk
    static constexpr int KPQ = 256 / LPK; // k-rows of B per load step
};

// TM = 128 (256 threads, two workgroups per CU) or 256 (512 threads, one
// workgroup per CU): each wave owns a 64 x 64 sub-tile either way; the taller
// tile reads its B chunk once for twice the rows.
template <typename T, int TAG, int RANGE, int TM = kTM>
__global__ void __launch_bounds__(2 * TM, 256 / TM) k_update(DevMesh dm, SysDesc sd, int e0, int ne, int k0, int KW,
                                                             int CB, int CW, int tiles_m, int tiles_n,
                                                             T *__restrict__ Ebase) {
    typedef UpdCfg<T> C;
    constexpr int NT = 2 * TM;                 // threads
    constexpr int RQ = NT / 8;                 // A-chunk rows per load step
    constexpr int KPQ = NT / C::LPK;           // B-chunk k-rows per load step
    constexpr int QB = C::KC / KPQ;            // B load steps per chunk
    static_assert(4 * RQ == TM && QB * KPQ == C::KC && QB >= 1, "update tile shape");
    typedef typename MF<T>::v16 v16;
    typedef typename MF<T>::acc_t acc_t;
    int el, t;
    if (!xcd_item(ne, tiles_m * tiles_n, el, t)) return;
    const int e = e0 + el;
    const ElemDims dd = elem_dims(dm, sd, e);
    if (k0 >= dd.n) return;
    const int rem = dd.n - k0;
    const int K = min(KW, rem);
    int rbeg, rend, cbeg, cend;
    if (RANGE == kRangeLU) {
        rbeg = k0 + K; rend = dd.mrows;
        cbeg = k0 + max(K, min(CB, rem));
        cend = CW > 0 ? k0 + min(CW, rem) : dd.ncols;
    } else {
        rbeg = k0 + K; rend = dd.n; cbeg = dd.n; cend = dd.ncols;
    }
    const int r0 = rbeg + (t / tiles_n) * TM;
    const int c0 = cbeg + (t % tiles_n) * kTN;
    if (r0 >= rend || c0 >= cend) return;
    T *E = Ebase + (sd.off[e] - sd.off[e0]);
    const int64_t ld = dd.ld;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;  // wave sub-tile origin
    __shared__ __attribute__((aligned(16))) T sA[2][TM][C::SA];
    __shared__ __attribute__((aligned(16))) T sB[2][C::KC][C::SB];
    // chunk loads with 16-byte accesses: A chunk (128 rows x KC k): 8 lanes per
    // 128-byte row segment, rows 32q + tid/8; B chunk (KC k x 128 columns): LPK
    // lanes per k-row of 1 KB (FP64) or 512 B (FP32).  Out-of-range entries are
    // read from a clamped in-range address and replaced by 0 (no branches): K and
    // every column offset are multiples of V, and a row holds ld >= ncols entries
    // with ld a multiple of 8.
    const int ar = tid >> 3, ak = (tid & 7) * C::V;
    const int bk = tid / C::LPK, bc = (tid % C::LPK) * C::V;
    const T *arow[4];
    bool aok[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int row = r0 + RQ * q + ar;
        aok[q] = row < rend;
        arow[q] = E + (int64_t)min(row, rend - 1) * ld + k0;
    }
    const int bcol = c0 + bc;
    const int bcolc = min(bcol, (cend - 1) & ~(C::V - 1));
    // The raw loads stay in registers while the current chunk's products run; the
    // out-of-range entries are zeroed only when the chunk is stored to LDS, so no
    // wait on the loads precedes the matrix-core work.
    auto load_chunk = [&](int kc, v16 *ra, v16 *rb) {
        const int gkc = min(kc + ak, (K - 1) & ~(C::V - 1));
#pragma unroll
        for (int q = 0; q < 4; ++q) ra[q] = *(const v16 *)(arow[q] + gkc);
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int gk2 = kc + KPQ * q + bk;
            rb[q] = *(const v16 *)(E + (int64_t)(k0 + min(gk2, K - 1)) * ld + bcolc);
        }
    };
    auto store_chunk = [&](int buf, int kc, const v16 *ra, const v16 *rb) {
        const int gk = kc + ak;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v16 a;
#pragma unroll
            for (int i = 0; i < C::V; ++i) a[i] = (aok[q] && gk + i < K) ? ra[q][i] : T(0);
            *(v16 *)&sA[buf][RQ * q + ar][ak] = (sizeof(T) == 8) ? -a : a;
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            v16 b;
            const int gk2 = kc + KPQ * q + bk;
            const bool k2ok = gk2 < K;
#pragma unroll
            for (int i = 0; i < C::V; ++i) b[i] = (k2ok && bcol + i < cend) ? rb[q][i] : T(0);
            *(v16 *)&sB[buf][KPQ * q + bk][bc] = b;
        }
    };
    // C is read at the start so that its loads overlap the operand loads.  FP64:
    // the accumulators start from C and A enters LDS negated (the epilogue only
    // stores).  FP32: C waits in registers of its own and the product is
    // accumulated from zero, so that every FP32 rounding stays at the scale of
    // the product rather than of C.
    constexpr bool kOntoC = sizeof(T) == 8;
    acc_t acc[4][4];
    acc_t cpre[kOntoC ? 1 : 4][4];
    const bool full = (r0 + TM <= rend) && (c0 + kTN <= cend);
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = r0 + wr + 16 * bi + MF<T>::rowof(lane, j);
            const T *row = E + (int64_t)min(r, rend - 1) * ld + c0 + wc + (lane & 15);
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) {
                const bool ok = full || (r < rend && c0 + wc + 16 * bj + (lane & 15) < cend);
                const T c = ok ? row[16 * bj] : T(0);
                if constexpr (kOntoC) {
                    acc[bi][bj][j] = c;
                } else {
                    cpre[bi][bj][j] = c;
                    acc[bi][bj][j] = T(0);
                }
            }
        }
    v16 ra[4], rb[QB];
    load_chunk(0, ra, rb);
    store_chunk(0, 0, ra, rb);
    __syncthreads();
    const int nchunks = (K + C::KC - 1) / C::KC;
    // a wave whose 64 x 64 sub-tile lies wholly outside the range (the other half
    // of a 64-column update, the rows past the end) only loads and synchronises,
    // leaving its SIMD's matrix core to the waves of the other workgroup
    const bool live = (r0 + wr < rend) && (c0 + wc < cend);  // uniform per wave
    for (int ch = 0; ch < nchunks; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nchunks) load_chunk((ch + 1) * C::KC, ra, rb);
        if (live) {
#pragma unroll
            for (int kk = 0; kk < C::KC; kk += 4) {
                T av[4], bv[4];
#pragma unroll
                for (int bi = 0; bi < 4; ++bi) av[bi] = sA[buf][wr + 16 * bi + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
                for (int bj = 0; bj < 4; ++bj) bv[bj] = sB[buf][kk + (lane >> 4)][wc + 16 * bj + (lane & 15)];
#pragma unroll
                for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                    for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = MF<T>::mfma(av[bi], bv[bj], acc[bi][bj]);
            }
        }
        if constexpr (!kOntoC) {
            // FP32: fold the partial product into C every kFold values of K, so the
            // rounding of each partial sum stays at the scale of 128 products
            if ((ch + 1) % (kFold / C::KC) == 0 && ch + 1 < nchunks) {
#pragma unroll
                for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                    for (int bj = 0; bj < 4; ++bj) {
                        cpre[bi][bj] -= acc[bi][bj];
                        acc[bi][bj] = (acc_t){T(0), T(0), T(0), T(0)};
                    }
            }
        }
        if (ch + 1 < nchunks) {
            store_chunk(buf ^ 1, (ch + 1) * C::KC, ra, rb);
            __syncthreads();
        }
    }
    // epilogue: C = C - A B
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = r0 + wr + 16 * bi + MF<T>::rowof(lane, j);
            T *row = E + (int64_t)r * ld + c0 + wc + (lane & 15);
            T v[4];
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) v[bj] = kOntoC ? acc[bi][bj][j] : cpre[kOntoC ? 0 : bi][bj][j] - acc[bi][bj][j];
            if (full) {
#pragma unroll
                for (int bj = 0; bj < 4; ++bj) row[16 * bj] = v[bj];
            } else if (r < rend) {
#pragma unroll
                for (int bj = 0; bj < 4; ++bj)
                    if (c0 + wc + 16 * bj + (lane & 15) < cend) row[16 * bj] = v[bj];
            }
        }
}

// ------------------------------------------------------------------ extract
// SK (column-major f x (f+1)) = [ trailing f x f block | - last column ]
template <typename T>
__global__ void __launch_bounds__(256) k_extract(DevMesh dm, SysDesc sd, int e0, const T *__restrict__ Ebase,
                                                 double *__restrict__ SK) {
    const int e = e0 + blockIdx.z;
    const ElemDims dd = elem_dims(dm, sd, e);
    const int f = dd.f;
    const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 32;  // i: row of S, j: column (0..f)
    if (i0 >= f || j0 > f) return;
    const T *E = Ebase + (sd.off[e] - sd.off[e0]);
    double *out = SK + dm.SK_off[e];
    __shared__ double tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int i = i0 + r, j = j0 + tx;
        double v = 0.0;
        if (i < f && j <= f) {
            v = (double)E[(int64_t)(dd.n + i) * dd.ld + dd.n + j];
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

// ------------------------------------------------------- back substitution
// Left-looking back substitution U X = Y on the right-hand columns n.., one
// 128-row block [k0, k0 + nb) per launch, the blocks below already solved:
// T = Y_blk - U[blk, k0+nb .. n) X[k0+nb .. n) on matrix cores (as k_update,
// with K = n - k0 - nb), then X_blk = U_blk^{-1} T with the recorded inverse
// [[Ua^{-1}, Uc], [0, Ub^{-1}]]: zero blocks skipped, wave w takes the 16-row
// blocks w and 7 - w (equal work), T passes through LDS in two 64-column
// halves.  One workgroup per (128-column tile, element), an element's tiles on
// one XCD.  In place.
template <typename T, int TAG>
__global__ void __launch_bounds__(256, 2) k_lbsolve(DevMesh dm, SysDesc sd, int e0, int ne, int k0, int tiles_n,
                                                    T *__restrict__ Ebase, WS<T> ws) {
    typedef UpdCfg<T> C;
    typedef typename MF<T>::v16 v16;
    typedef typename MF<T>::acc_t acc_t;
    int el, tl;
    if (!xcd_item(ne, tiles_n, el, tl)) return;
    const int e = e0 + el;
    const ElemDims dd = elem_dims(dm, sd, e);
    if (k0 >= dd.n) return;
    const int nb = min(kNBO, dd.n - k0);
    const int kb = k0 + nb;  // first row (and column) of the solved part
    const int K = dd.n - kb;
    const int r0 = k0, rend = kb;
    const int c0 = dd.n + tl * kTN, cend = dd.ncols;
    if (c0 >= cend) return;  // uniform per block
    T *E = Ebase + (sd.off[e] - sd.off[e0]);
    const T *wd = ws.d + (int64_t)el * ws.ds;
    const int64_t ld = dd.ld;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
    // LDS: the double-buffered operand chunks, later the 128 x 64 half of T
    constexpr int kStageA = 2 * kTM * C::SA, kStageB = 2 * C::KC * C::SB, kHalfT = kNBO * 65;
    constexpr int kWords = (kStageA + kStageB > kHalfT) ? kStageA + kStageB : kHalfT;
    __shared__ __attribute__((aligned(16))) T smem[kWords];
    T (*sA)[kTM][C::SA] = reinterpret_cast<T (*)[kTM][C::SA]>(smem);
    T (*sB)[C::KC][C::SB] = reinterpret_cast<T (*)[C::KC][C::SB]>(smem + kStageA);
    T (*sT)[65] = reinterpret_cast<T (*)[65]>(smem);
    const int ar = tid >> 3, ak = (tid & 7) * C::V;
    const int bk = tid / C::LPK, bc = (tid % C::LPK) * C::V;
    // T = Y - U_right X_below: operands as in k_update (16-byte loads from clamped
    // in-range addresses, out-of-range entries replaced by 0; K and the column
    // offsets are multiples of V)
    constexpr bool kOntoC = sizeof(T) == 8;
    acc_t acc[4][4];
    acc_t cpre[kOntoC ? 1 : 4][4];
    const bool full = (r0 + kTM <= rend) && (c0 + kTN <= cend);
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = r0 + wr + 16 * bi + MF<T>::rowof(lane, j);
            const T *row = E + (int64_t)min(r, rend - 1) * ld + c0 + wc + (lane & 15);
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) {
                const bool ok = full || (r < rend && c0 + wc + 16 * bj + (lane & 15) < cend);
                const T c = ok ? row[16 * bj] : T(0);
                if constexpr (kOntoC) {
                    acc[bi][bj][j] = c;
                } else {
                    cpre[bi][bj][j] = c;
                    acc[bi][bj][j] = T(0);
                }
            }
        }
    if (K > 0) {
        const T *arow[4];
        bool aok[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = r0 + 32 * q + ar;
            aok[q] = row < rend;
            arow[q] = E + (int64_t)min(row, rend - 1) * ld + kb;
        }
        const int bcol = c0 + bc;
        const int bcolc = min(bcol, (cend - 1) & ~(C::V - 1));
        // raw loads in registers; out-of-range entries zeroed at the LDS store
        auto load_chunk = [&](int kc, v16 *ra, v16 *rb) {
            const int gkc = min(kc + ak, (K - 1) & ~(C::V - 1));
#pragma unroll
            for (int q = 0; q < 4; ++q) ra[q] = *(const v16 *)(arow[q] + gkc);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int gk2 = kc + C::KPQ * q + bk;
                rb[q] = *(const v16 *)(E + (int64_t)(kb + min(gk2, K - 1)) * ld + bcolc);
            }
        };
        auto store_chunk = [&](int buf, int kc, const v16 *ra, const v16 *rb) {
            const int gk = kc + ak;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                v16 a, b;
                const int gk2 = kc + C::KPQ * q + bk;
                const bool k2ok = gk2 < K;
#pragma unroll
                for (int i = 0; i < C::V; ++i) {
                    a[i] = (aok[q] && gk + i < K) ? ra[q][i] : T(0);
                    b[i] = (k2ok && bcol + i < cend) ? rb[q][i] : T(0);
                }
                *(v16 *)&sA[buf][32 * q + ar][ak] = kOntoC ? -a : a;
                *(v16 *)&sB[buf][C::KPQ * q + bk][bc] = b;
            }
        };
        v16 ra[4], rb[4];
        load_chunk(0, ra, rb);
        store_chunk(0, 0, ra, rb);
        __syncthreads();
        const int nchunks = (K + C::KC - 1) / C::KC;
        for (int ch = 0; ch < nchunks; ++ch) {
            const int buf = ch & 1;
            if (ch + 1 < nchunks) load_chunk((ch + 1) * C::KC, ra, rb);
#pragma unroll
            for (int kk = 0; kk < C::KC; kk += 4) {
                T av[4], bv[4];
#pragma unroll
                for (int bi = 0; bi < 4; ++bi) av[bi] = sA[buf][wr + 16 * bi + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
                for (int bj = 0; bj < 4; ++bj) bv[bj] = sB[buf][kk + (lane >> 4)][wc + 16 * bj + (lane & 15)];
#pragma unroll
                for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                    for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = MF<T>::mfma(av[bi], bv[bj], acc[bi][bj]);
            }
            if constexpr (!kOntoC) {
                // FP32: fold the partial product into Y every kFold values of K
                if ((ch + 1) % (kFold / C::KC) == 0 && ch + 1 < nchunks) {
#pragma unroll
                    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                        for (int bj = 0; bj < 4; ++bj) {
                            cpre[bi][bj] -= acc[bi][bj];
                            acc[bi][bj] = (acc_t){T(0), T(0), T(0), T(0)};
                        }
                }
            }
            if (ch + 1 < nchunks) {
                store_chunk(buf ^ 1, (ch + 1) * C::KC, ra, rb);
                __syncthreads();
            }
        }
    }
    if constexpr (!kOntoC) {
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = cpre[bi][bj] - acc[bi][bj];
    }
    // X_blk = U_blk^{-1} T, 64 columns at a time (rows >= nb of T are zero)
    const int kq = lane >> 4, cl = lane & 15;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        __syncthreads();
        if (wc == 64 * h) {
#pragma unroll
            for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                for (int bj = 0; bj < 4; ++bj)
#pragma unroll
                    for (int j = 0; j < 4; ++j) sT[wr + 16 * bi + MF<T>::rowof(lane, j)][16 * bj + cl] = acc[bi][bj][j];
        }
        __syncthreads();
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            const int rb = hh == 0 ? wave : 7 - wave;
            if (16 * rb >= nb) continue;  // uniform per wave
            acc_t o[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) o[j] = (acc_t){T(0), T(0), T(0), T(0)};
            const int r = 16 * rb + cl;
            if (rb < 4) {
                mfma_rowblock<T, 4>(wd + 2 * kNB * kNB + r * kNB + kq, sT, 0, 16 * rb, kNB, kq, cl, o);  // Ua^{-1}
                if (nb > kNB) mfma_rowblock<T, 4>(wd + kWsUc + r * kNB + kq, sT, kNB, 0, kNB, kq, cl, o);  // Uc
            } else {
                mfma_rowblock<T, 4>(wd + 3 * kNB * kNB + (r - kNB) * kNB + kq, sT, kNB, 16 * (rb - 4), kNB, kq, cl,
                                    o);  // Ub^{-1}
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int rr = 16 * rb + MF<T>::rowof(lane, q), c = c0 + 64 * h + 16 * j + cl;
                    if (rr < nb && c < cend) E[(int64_t)(k0 + rr) * ld + c] = o[j][q];
                }
        }
    }
}

// ---------------------------------------------------- mixed precision only
__device__ inline void mixed_dims(const DevMesh &dm, int e, int &n, int &f, int64_t &ld, int64_t &ldx) {
    const int p = dm.elem_p[e];
    n = 20 * (p + 1) * (p + 1) * (p + 1);
    f = dm.toff[7 * e + 6];
    ld = e_ld(n, f);
    ldx = x_ld(f);
}

// FP32 copy of the interior rows [A | B R_qu] (padding columns included).
__global__ void __launch_bounds__(256) k_to32(DevMesh dm, int e0, const double *__restrict__ Ebase,
                                              float *__restrict__ Mbase) {
    const int e = e0 + blockIdx.y;
    int n, f;
    int64_t ld, ldx;
    mixed_dims(dm, e, n, f, ld, ldx);
    const MF<double>::v2 *E = (const MF<double>::v2 *)(Ebase + (dm.E_off[e] - dm.E_off[e0]));
    MF<float>::v2 *M = (MF<float>::v2 *)(Mbase + (dm.m32_off[e] - dm.m32_off[e0]));
    const int64_t total = (int64_t)n * ld / 2;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const MF<double>::v2 v = E[i];
        M[i] = (MF<float>::v2){(float)v.x, (float)v.y};
    }
}

// X (FP64, n x x_ld) = the right-hand columns of the FP32 system (MODE 0), or
// X += them (MODE 1), or X += them and X is also written into E's [B | R_qu]
// columns (MODE 2, the last refinement step).
template <int MODE>
__global__ void __launch_bounds__(256) k_xupdate(DevMesh dm, int e0, const float *__restrict__ Mbase,
                                                 double *__restrict__ Xbase, double *__restrict__ Ebase) {
    const int e = e0 + blockIdx.y;
    int n, f;
    int64_t ld, ldx;
    mixed_dims(dm, e, n, f, ld, ldx);
    const float *M = Mbase + (dm.m32_off[e] - dm.m32_off[e0]);
    double *X = Xbase + (dm.x_off[e] - dm.x_off[e0]);
    double *E = Ebase + (dm.E_off[e] - dm.E_off[e0]);
    for (int r = blockIdx.x; r < n; r += gridDim.x)
        for (int c = threadIdx.x; c < ldx; c += 256) {
            const double m = (c <= f) ? (double)M[(int64_t)r * ld + n + c] : 0.0;
            const int64_t i = (int64_t)r * ldx + c;
            const double x = (MODE == 0) ? m : X[i] + m;
            X[i] = x;
            if (MODE == 2 && c <= f) E[(int64_t)r * ld + n + c] = x;
        }
}

// Column fields of A that can be nonzero in row field fr (fields: q_(c,j) = 3c+j,
// u_c = 15+c).  R_q couples q_(c,j) to itself (mass) and to u_c; R_u couples
// u_c to every u (convective, viscous, mass and tau terms) and to the gradients
// its fluxes read: the artificial viscosity term only for c = 0, the velocity
// gradients (q of c' = 0..3) for the momentum rows, all of q for the energy row.
__device__ inline unsigned a_field_mask(int fr) {
    if (fr < 15) return (1u << fr) | (1u << (15 + fr / 3));
    const unsigned u = 0x1Fu << 15;
    const int c = fr - 15;
    return c == 0 ? (u | 0x7u) : (c == 4 ? (u | 0x7FFFu) : (u | 0xFFFu));
}

// FP64 products of the mixed path, 128 x 128 tiles on FP64 matrix cores:
//   OP 0 (refinement residual): R = [B | R_qu] - A X over rows 0..n-1, stored in
//        FP32 into the right-hand columns of the FP32 system.  K chunks whose
//        column fields are structurally zero in every row field of the tile are
//        skipped (those entries of A are exact zeros).
//   OP 1 (Schur complement): [S^K | -g^K] = [D | R_uh] - C X over rows n..n+f-1,
//        written to SK column-major with the last column negated.
template <int OP>
__global__ void __launch_bounds__(256, 2) k_gemm64(DevMesh dm, int e0, int ne, int tiles_m, int tiles_n,
                                                   const double *__restrict__ Ebase, const double *__restrict__ Xbase,
                                                   float *__restrict__ Mbase, double *__restrict__ SK) {
    typedef UpdCfg<double> C;
    typedef MF<double>::v16 v16;
    typedef MF<double>::acc_t acc_t;
    int el, t;
    if (!xcd_item(ne, tiles_m * tiles_n, el, t)) return;
    const int e = e0 + el;
    int n, f;
    int64_t ld, ldx;
    mixed_dims(dm, e, n, f, ld, ldx);
    const int Mrows = (OP == 0) ? n : f, N = f + 1, K = n;
    const int r0 = (t / tiles_n) * kTM, c0 = (t % tiles_n) * kTN;
    if (r0 >= Mrows || c0 >= N) return;
    const int arow0 = (OP == 0) ? 0 : n;
    const double *E = Ebase + (dm.E_off[e] - dm.E_off[e0]);
    const double *X = Xbase + (dm.x_off[e] - dm.x_off[e0]);
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
    __shared__ __attribute__((aligned(16))) double sA[2][kTM][C::SA];
    __shared__ __attribute__((aligned(16))) double sB[2][C::KC][C::SB];
    const int ar = tid >> 3, ak = (tid & 7) * C::V;
    const int bk = tid / C::LPK, bc = (tid % C::LPK) * C::V;
    const double *arow[4];
    bool aok[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int row = r0 + 32 * q + ar;
        aok[q] = row < Mrows;
        arow[q] = E + (int64_t)(arow0 + min(row, Mrows - 1)) * ld;
    }
    const int bcol = c0 + bc;
    const int bcolc = min(bcol, (N - 1) & ~1);
    // raw loads in registers; out-of-range entries zeroed at the LDS store
    auto load_chunk = [&](int kc, v16 *ra, v16 *rb) {
        const int gkc = min(kc + ak, (K - 1) & ~1);
#pragma unroll
        for (int q = 0; q < 4; ++q) ra[q] = *(const v16 *)(arow[q] + gkc);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int gk2 = kc + C::KPQ * q + bk;
            rb[q] = *(const v16 *)(X + (int64_t)min(gk2, K - 1) * ldx + bcolc);
        }
    };
    auto store_chunk = [&](int buf, int kc, const v16 *ra, const v16 *rb) {
        const int gk = kc + ak;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v16 a, b;
            const int gk2 = kc + C::KPQ * q + bk;
            const bool k2ok = gk2 < K;
            a.x = (aok[q] && gk < K) ? ra[q].x : 0.0;
            a.y = (aok[q] && gk + 1 < K) ? ra[q].y : 0.0;
            b.x = (k2ok && bcol < N) ? rb[q].x : 0.0;
            b.y = (k2ok && bcol + 1 < N) ? rb[q].y : 0.0;
            *(v16 *)&sA[buf][32 * q + ar][ak] = a;
            *(v16 *)&sB[buf][C::KPQ * q + bk][bc] = b;
        }
    };
    // K chunks this tile needs
    const int Np = n / 20;
    unsigned rmask = 0xFFFFFu;
    if (OP == 0) {
        rmask = 0;
        const int fr1 = (min(r0 + kTM, Mrows) - 1) / Np;
        for (int fr = r0 / Np; fr <= fr1; ++fr) rmask |= a_field_mask(fr);
    }
    const int nchunks = (K + C::KC - 1) / C::KC;
    auto needed = [&](int ch) {
        const int k_lo = ch * C::KC, k_hi = min(k_lo + C::KC, K) - 1;
        const int f0 = k_lo / Np, f1 = k_hi / Np;
        const unsigned span = ((2u << f1) - 1u) & ~((1u << f0) - 1u);
        return (rmask & span) != 0u;
    };
    auto next_needed = [&](int ch) {
        while (ch < nchunks && !needed(ch)) ++ch;
        return ch;
    };
    // the same test per 16-row block of this wave (uniform per wave): a block
    // skips the products of a chunk whose columns are zero in all its rows
    unsigned bmask[4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) {
        const int lo = r0 + wr + 16 * bi, hi = min(lo + 15, Mrows - 1);
        bmask[bi] = 0;
        if (OP != 0) bmask[bi] = 0xFFFFFu;
        else if (lo < Mrows)
            for (int fr = lo / Np; fr <= hi / Np; ++fr) bmask[bi] |= a_field_mask(fr);
    }
    acc_t acc[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = (acc_t){0.0, 0.0, 0.0, 0.0};
    v16 ra[4], rb[4];
    int ch = next_needed(0);
    int buf = 0;
    if (ch < nchunks) {
        load_chunk(ch * C::KC, ra, rb);
        store_chunk(0, ch * C::KC, ra, rb);
        __syncthreads();
    }
    while (ch < nchunks) {
        const int nx = next_needed(ch + 1);
        if (nx < nchunks) load_chunk(nx * C::KC, ra, rb);
        bool use[4];
        {
            const int k_lo = ch * C::KC, k_hi = min(k_lo + C::KC, K) - 1;
            const unsigned span = ((2u << (k_hi / Np)) - 1u) & ~((1u << (k_lo / Np)) - 1u);
#pragma unroll
            for (int bi = 0; bi < 4; ++bi) use[bi] = (bmask[bi] & span) != 0u;
        }
#pragma unroll
        for (int kk = 0; kk < C::KC; kk += 4) {
            double av[4], bv[4];
#pragma unroll
            for (int bi = 0; bi < 4; ++bi) av[bi] = sA[buf][wr + 16 * bi + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) bv[bj] = sB[buf][kk + (lane >> 4)][wc + 16 * bj + (lane & 15)];
#pragma unroll
            for (int bi = 0; bi < 4; ++bi)
                if (use[bi])
#pragma unroll
                    for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = MF<double>::mfma(av[bi], bv[bj], acc[bi][bj]);
        }
        if (nx < nchunks) {
            store_chunk(buf ^ 1, nx * C::KC, ra, rb);
            __syncthreads();
        }
        buf ^= 1;
        ch = nx;
    }
    // epilogue: out = Cin - product; the 16 Cin values of a row block are loaded
    // together from clamped in-range addresses before any of them is used
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) {
        double cv[4][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = min(r0 + wr + 16 * bi + MF<double>::rowof(lane, j), Mrows - 1);
            const double *cin = E + (int64_t)(arow0 + r) * ld + n;
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) cv[j][bj] = cin[min(c0 + wc + 16 * bj + (lane & 15), N - 1)];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = r0 + wr + 16 * bi + MF<double>::rowof(lane, j);
            if (r >= Mrows) continue;
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) {
                const int c = c0 + wc + 16 * bj + (lane & 15);
                if (c >= N) continue;
                const double v = cv[j][bj] - acc[bi][bj][j];
                if (OP == 0) {
                    float *M = Mbase + (dm.m32_off[e] - dm.m32_off[e0]);
                    M[(int64_t)r * ld + n + c] = (float)v;
                } else {
                    SK[dm.SK_off[e] + (int64_t)c * f + r] = (c == f) ? -v : v;
                }
            }
        }
    }
}

}  // namespace

// Rows of the trailing-update tile for systems with n pivot columns: the
// context's setting for that n (hdg_set_update_tile), else for every n, else 128.
static int update_tile_rows(const hdg_ctx *ctx, int n) {
    auto it = ctx->update_tile.find(n);
    if (it != ctx->update_tile.end()) return it->second;
    it = ctx->update_tile.find(0);
    return it != ctx->update_tile.end() ? it->second : kTM;
}

// Blocked LU of the systems e0..e0+ne-1 described by sd (bordered: trace rows
// included when maxf_rows > 0).  ws: per-element workspace of a pair of
// 128-column blocks, or with `persist` one per block (ws strides hold all of
// them).  maxc: most columns of a system; maxrhs: most columns right of the n
// pivot columns.
//
// The blocks go in pairs (A at K0, B at K0 + 128) so that the columns beyond
// the pair receive one update with K = 256 instead of two with K = 128, which
// halves the traffic of the trailing matrix:
//   factor A; U rows and update of B's columns by A only; factor B;
//   B's swaps on A's L; A's U rows on the far columns; B's U rows on the far
//   columns (A's update applied to B's gathered rows); far update, K = 256.
template <typename T, int TAG>
static int run_lu(const hdg_ctx *ctx, const SysDesc &sd, int e0, int ne, T *E, int *info, WS<T> ws, bool persist,
                  int maxn, int maxm, int maxc, int maxrhs, int maxf_rows, hipStream_t s) {
    const DevMesh &dm = ctx->dm;
    hipLaunchKernelGGL(k_zero_int, dim3((ne + 255) / 256), dim3(256), 0, s, info + e0, ne);
    const int R = (maxn + kPT - 1) / kPT;
    if (R > 5) return (int)hipErrorInvalidValue;
    auto block_ws_of = [&](int bi) {
        WS<T> wb = ws;
        const int slot = persist ? bi : (bi & 1);
        wb.d += (int64_t)slot * kWsDbl;
        wb.i += (int64_t)slot * kWsInt;
        return wb;
    };
    const int TMr = update_tile_rows(ctx, maxn);
    auto update = [&](int k0, int KW, int CB, int CW, int rows, int cols) {
        if (rows <= 0 || cols <= 0) return;
        const int tm = (rows + TMr - 1) / TMr, tn = (cols + kTN - 1) / kTN;
        if (TMr == 256)
            hipLaunchKernelGGL((k_update<T, TAG, kRangeLU, 256>), dim3(xcd_grid(ne, tm * tn)), dim3(512), 0, s, dm, sd,
                               e0, ne, k0, KW, CB, CW, tm, tn, E);
        else
            hipLaunchKernelGGL((k_update<T, TAG, kRangeLU>), dim3(xcd_grid(ne, tm * tn)), dim3(256), 0, s, dm, sd, e0,
                               ne, k0, KW, CB, CW, tm, tn, E);
    };
    auto blocku = [&](auto mode, int k0, const WS<T> &wb, int CB, int CW, int cols) {
        if (cols <= 0) return;
        const int tiles = (cols + kBC - 1) / kBC;
        hipLaunchKernelGGL((k_blocku<decltype(mode)::value, TAG, T>), dim3(xcd_grid(ne, tiles)), dim3(256), 0, s,
                           dm, sd, e0, ne, k0, 0, CB, CW, tiles, E, wb);
    };
    // panels of the 128-column block at k0 and their records
    auto factor_block = [&](int k0, const WS<T> &wb) {
        auto panel = [&](int kp, int slot) {
            auto half = [&](int part) {
                if (R <= 1) hipLaunchKernelGGL((k_panel<1, TAG, T>), dim3(ne), dim3(kPT), 0, s, dm, sd, e0, kp, slot, k0, part, E, wb, info);
                else if (R <= 2) hipLaunchKernelGGL((k_panel<2, TAG, T>), dim3(ne), dim3(kPT), 0, s, dm, sd, e0, kp, slot, k0, part, E, wb, info);
                else if (R <= 3) hipLaunchKernelGGL((k_panel<3, TAG, T>), dim3(ne), dim3(kPT), 0, s, dm, sd, e0, kp, slot, k0, part, E, wb, info);
                else hipLaunchKernelGGL((k_panel<5, TAG, T>), dim3(ne), dim3(kPT), 0, s, dm, sd, e0, kp, slot, k0, part, E, wb, info);
            };
            half(1);
            if (maxn - kp > kHalf)
                hipLaunchKernelGGL((k_half<TAG, T>), dim3((maxn - kp - kHalf + 63) / 64, ne), dim3(256), 0, s, dm, sd, e0,
                                   kp, E);
            half(2);
            if (maxf_rows > 0)
                hipLaunchKernelGGL((k_crows<TAG, T>), dim3((maxf_rows + kCR - 1) / kCR, ne), dim3(256), 0, s, dm, sd, e0,
                                   kp, slot, E, wb);
        };
        panel(k0, 0);
        if (maxn - k0 > kNB) {
            // rest of the 128-column block, then its second panel
            hipLaunchKernelGGL((k_rowperm<0, TAG, T>), dim3(kNB / kRPC, ne), dim3(256), 0, s, dm, sd, e0, k0, kNBO, E, wb);
            update(k0, kNB, 0, kNBO, maxm - k0, kNB);
            panel(k0 + kNB, 1);
            hipLaunchKernelGGL((k_rowperm<1, TAG, T>), dim3(kNB / kRPC, ne), dim3(256), 0, s, dm, sd, e0, k0, 0, E, wb);
            hipLaunchKernelGGL((k_inv128<TAG, T>), dim3(ne), dim3(256), 0, s, dm, sd, e0, k0, (const T *)E, wb);
        }
    };
    using M0 = std::integral_constant<int, 0>;
    using M1 = std::integral_constant<int, 1>;
    using M2 = std::integral_constant<int, 2>;
    for (int K0 = 0, pi = 0; K0 < maxn; K0 += 2 * kNBO, ++pi) {
        const WS<T> wa = block_ws_of(2 * pi), wb = block_ws_of(2 * pi + 1);
        const bool pairB = maxn - K0 > kNBO;
        factor_block(K0, wa);
        if (pairB) {
            blocku(M0{}, K0, wa, 0, 2 * kNBO, kNBO);
            update(K0, kNBO, 0, 2 * kNBO, maxm - K0, kNBO);
            factor_block(K0 + kNBO, wb);
            blocku(M2{}, K0 + kNBO, wb, 0, 0, kNBO);
        }
        // far columns: beyond the pair (the right-hand and trace columns included)
        const int far = std::max(maxc - K0 - 2 * kNBO, maxrhs);
        blocku(M0{}, K0, wa, 2 * kNBO, 0, far);
        if (pairB) blocku(M1{}, K0 + kNBO, wb, kNBO, 0, far);
        update(K0, 2 * kNBO, 2 * kNBO, 0, maxm - K0, far);
    }
    return (int)hipGetLastError();
}

static void chunk_max(const hdg_ctx *ctx, int e0, int ne, int *maxn, int *maxf) {
    *maxn = 0;
    *maxf = 0;
    for (int e = e0; e < e0 + ne; ++e) {
        *maxn = std::max(*maxn, ctx->elem_n[e]);
        *maxf = std::max(*maxf, ctx->elem_f[e]);
    }
}

int launch_condense_fp64(const hdg_ctx *ctx, int e0, int ne, double *E, double *SK, int *info, void *work,
                         hipStream_t s) {
    int maxn, maxf, maxm = 0;
    chunk_max(ctx, e0, ne, &maxn, &maxf);
    for (int e = e0; e < e0 + ne; ++e) maxm = std::max(maxm, ctx->elem_n[e] + ctx->elem_f[e]);
    const SysDesc sd{0, ctx->dm.E_off};
    WS<double> ws{(double *)work, (int *)((char *)work + sizeof(double) * (size_t)ne * 2 * kWsDbl), 2 * kWsDbl,
                  2 * kWsInt};
    int err = run_lu<double, 0>(ctx, sd, e0, ne, E, info, ws, false, maxn, maxm, maxm + 1, maxf + 1, maxf, s);
    if (err) return err;
    hipLaunchKernelGGL(k_extract<double>, dim3((maxf + 1 + 31) / 32, (maxf + 31) / 32, ne), dim3(256), 0, s,
                       ctx->dm, sd, e0, (const double *)E, SK);
    return (int)hipGetLastError();
}

size_t bordered_lu_work(const hdg_ctx *ctx, int ne) {
    (void)ctx;
    return 2 * (sizeof(double) * (size_t)ne * kWsDbl + sizeof(int) * (size_t)ne * kWsInt);
}

template <typename T> static WS<T> block_ws(WS<T> ws, int k0) {
    ws.d += (int64_t)(k0 / kNBO) * kWsDbl;
    ws.i += (int64_t)(k0 / kNBO) * kWsInt;
    return ws;
}

// Back substitution U X = Y on the right-hand columns n .. ncols of factored
// systems (the per-block records in ws kept by run_lu with persist), in place,
// from the last 128-row block up.
template <typename T, int TAG>
static void run_back_solve(const hdg_ctx *ctx, const SysDesc &sd, int e0, int ne, T *E, WS<T> ws, int maxn,
                           int rhs_cols, hipStream_t s) {
    const DevMesh &dm = ctx->dm;
    const int tn = (rhs_cols + kTN - 1) / kTN;
    for (int k0 = (maxn - 1) / kNBO * kNBO; k0 >= 0; k0 -= kNBO)
        hipLaunchKernelGGL((k_lbsolve<T, TAG>), dim3(xcd_grid(ne, tn)), dim3(256), 0, s, dm, sd, e0, ne, k0, tn, E,
                           block_ws(ws, k0));
}

// Forward substitution L Y = P R of new right-hand columns, replaying the
// recorded permutations and the pairing of the blocks as the factorisation did.
template <typename T, int TAG>
static void run_forward_solve(const hdg_ctx *ctx, const SysDesc &sd, int e0, int ne, T *E, WS<T> ws, int maxn,
                              int rhs_cols, hipStream_t s) {
    const DevMesh &dm = ctx->dm;
    const int tn = (rhs_cols + kTN - 1) / kTN;
    const int tiles = (rhs_cols + kBC - 1) / kBC;
    for (int K0 = 0; K0 < maxn; K0 += 2 * kNBO) {
        hipLaunchKernelGGL((k_blocku<0, TAG, T>), dim3(xcd_grid(ne, tiles)), dim3(256), 0, s, dm, sd, e0, ne, K0, 1,
                           0, 0, tiles, E, block_ws(ws, K0));
        if (maxn - K0 > kNBO)
            hipLaunchKernelGGL((k_blocku<1, TAG, T>), dim3(xcd_grid(ne, tiles)), dim3(256), 0, s, dm, sd, e0, ne,
                               K0 + kNBO, 1, 0, 0, tiles, E, block_ws(ws, K0 + kNBO));
        const int rows = maxn - K0 - 2 * kNBO;
        if (rows > 0) {
            const int TMr = update_tile_rows(ctx, maxn);
            const int tm = (rows + TMr - 1) / TMr;
            if (TMr == 256)
                hipLaunchKernelGGL((k_update<T, TAG, kRangeFwd, 256>), dim3(xcd_grid(ne, tm * tn)), dim3(512), 0, s, dm,
                                   sd, e0, ne, K0, 2 * kNBO, 0, 0, tm, tn, E);
            else
                hipLaunchKernelGGL((k_update<T, TAG, kRangeFwd>), dim3(xcd_grid(ne, tm * tn)), dim3(256), 0, s, dm, sd,
                                   e0, ne, K0, 2 * kNBO, 0, 0, tm, tn, E);
        }
    }
}

// Schwarz blocks: systems [S_r | I] in `sys` (offsets asmsys_off, FP64 or FP32
// entries): LU with partial pivoting, then back substitution on the identity
// columns, which then hold S_r^{-1}.
static int schwarz_nblk(const hdg_ctx *ctx) { return std::max(1, (asm_pad(ctx->max_f) + kNBO - 1) / kNBO); }

size_t schwarz_ws_bytes(const hdg_ctx *ctx, int prec) {
    const size_t es = (prec == HDG_FP64) ? sizeof(double) : sizeof(float);
    const size_t per = (size_t)schwarz_nblk(ctx) * ((size_t)kWsDbl * es + (size_t)kWsInt * sizeof(int));
    return per * (size_t)ctx->n_elem + 256;
}

int run_asm_inversion(const hdg_ctx *ctx, int prec, void *sys, int *info, void *iwork, hipStream_t s) {
    const SysDesc sd{1, ctx->dm.asmsys_off};
    const int m = asm_pad(ctx->max_f);
    const int ne = ctx->n_elem;
    const int nblk = schwarz_nblk(ctx);
    const size_t es = (prec == HDG_FP64) ? sizeof(double) : sizeof(float);
    int *wi = (int *)((char *)iwork + ((es * (size_t)ne * nblk * kWsDbl + 255) / 256 * 256));
    if (prec == HDG_FP64) {
        WS<double> ws{(double *)iwork, wi, (int64_t)nblk * kWsDbl, (int64_t)nblk * kWsInt};
        int err = run_lu<double, 1>(ctx, sd, 0, ne, (double *)sys, info, ws, true, m, m, 2 * m + 1, m + 1, 0, s);
        if (err) return err;
        run_back_solve<double, 1>(ctx, sd, 0, ne, (double *)sys, ws, m, m + 1, s);
    } else {
        WS<float> ws{(float *)iwork, wi, (int64_t)nblk * kWsDbl, (int64_t)nblk * kWsInt};
        int err = run_lu<float, 3>(ctx, sd, 0, ne, (float *)sys, info, ws, true, m, m, 2 * m + 1, m + 1, 0, s);
        if (err) return err;
        run_back_solve<float, 3>(ctx, sd, 0, ne, (float *)sys, ws, m, m + 1, s);
    }
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------- mixed path
// Workspace of a chunk: FP32 systems | X (FP64) | per-block LU records (FP32 values, ints).
struct MixedLayout {
    size_t m_off, x_off, wd_off, wi_off, total;
    int nblk;
};
static size_t r256(size_t b) { return (b + 255) / 256 * 256; }
static MixedLayout mixed_layout(const hdg_ctx *ctx, int e0, int ne) {
    int maxn, maxf;
    chunk_max(ctx, e0, ne, &maxn, &maxf);
    MixedLayout L;
    L.nblk = std::max(1, (maxn + kNBO - 1) / kNBO);
    L.m_off = 0;
    L.x_off = L.m_off + r256(sizeof(float) * (size_t)(ctx->m32_off[e0 + ne] - ctx->m32_off[e0]));
    L.wd_off = L.x_off + r256(sizeof(double) * (size_t)(ctx->x_off[e0 + ne] - ctx->x_off[e0]));
    L.wi_off = L.wd_off + r256(sizeof(float) * (size_t)ne * L.nblk * kWsDbl);
    L.total = L.wi_off + r256(sizeof(int) * (size_t)ne * L.nblk * kWsInt);
    return L;
}

size_t condense_mixed_work_bytes(const hdg_ctx *ctx, int e0, int ne) { return mixed_layout(ctx, e0, ne).total; }

// ------------------------------------------------ all-FP32 variant (reported)
// The whole bordered element system in FP32 (E_off offsets, counted in floats),
// factored by the same blocked LU with FP32 matrix cores: its trailing updates
// form S^K and -g^K in FP32 (no refinement, FP32 Schur products).  Afterwards
// the interior rows (U, L^{-1} P [B | R_qu]) go back to E in FP64 for the
// recovery.
__global__ void __launch_bounds__(256) k_full_to32(DevMesh dm, int e0, const double *__restrict__ Ebase,
                                                   float *__restrict__ Fbase) {
    const int e = e0 + blockIdx.y;
    const int64_t o = dm.E_off[e] - dm.E_off[e0], total = dm.E_off[e + 1] - dm.E_off[e];
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256)
        Fbase[o + i] = (float)Ebase[o + i];
}
__global__ void __launch_bounds__(256) k_interior_to64(DevMesh dm, int e0, const float *__restrict__ Fbase,
                                                       double *__restrict__ Ebase) {
    const int e = e0 + blockIdx.y;
    const int p = dm.elem_p[e], n = 20 * (p + 1) * (p + 1) * (p + 1), f = dm.toff[7 * e + 6];
    const int64_t o = dm.E_off[e] - dm.E_off[e0], total = (int64_t)n * e_ld(n, f);
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256)
        Ebase[o + i] = (double)Fbase[o + i];
}

size_t condense_fast_work_bytes(const hdg_ctx *ctx, int e0, int ne) {
    const size_t sys = r256(sizeof(float) * (size_t)(ctx->E_off[e0 + ne] - ctx->E_off[e0]));
    return sys + r256(2 * (sizeof(float) * (size_t)ne * kWsDbl)) + r256(2 * sizeof(int) * (size_t)ne * kWsInt);
}

int launch_condense_fast(const hdg_ctx *ctx, int e0, int ne, double *E, double *SK, int *info, void *work,
                         hipStream_t s) {
    int maxn, maxf, maxm = 0;
    chunk_max(ctx, e0, ne, &maxn, &maxf);
    for (int e = e0; e < e0 + ne; ++e) maxm = std::max(maxm, ctx->elem_n[e] + ctx->elem_f[e]);
    char *wb = (char *)work;
    float *F = (float *)wb;
    const size_t sys = r256(sizeof(float) * (size_t)(ctx->E_off[e0 + ne] - ctx->E_off[e0]));
    float *wd = (float *)(wb + sys);
    int *wi = (int *)(wb + sys + r256(2 * (sizeof(float) * (size_t)ne * kWsDbl)));
    const SysDesc sd{0, ctx->dm.E_off};
    WS<float> ws{wd, wi, 2 * kWsDbl, 2 * kWsInt};
    const dim3 grid(64, ne);
    hipLaunchKernelGGL(k_full_to32, grid, dim3(256), 0, s, ctx->dm, e0, (const double *)E, F);
    int err = run_lu<float, 4>(ctx, sd, e0, ne, F, info, ws, false, maxn, maxm, maxm + 1, maxf + 1, maxf, s);
    if (err) return err;
    hipLaunchKernelGGL(k_extract<float>, dim3((maxf + 1 + 31) / 32, (maxf + 31) / 32, ne), dim3(256), 0, s,
                       ctx->dm, sd, e0, (const float *)F, SK);
    hipLaunchKernelGGL(k_interior_to64, grid, dim3(256), 0, s, ctx->dm, e0, (const float *)F, E);
    return (int)hipGetLastError();
}

int launch_condense_mixed(const hdg_ctx *ctx, int e0, int ne, int refine, double *E, double *SK, int *info,
                          void *work, hipStream_t s) {
    const DevMesh &dm = ctx->dm;
    int maxn, maxf;
    chunk_max(ctx, e0, ne, &maxn, &maxf);
    const MixedLayout L = mixed_layout(ctx, e0, ne);
    char *wb = (char *)work;
    float *M = (float *)(wb + L.m_off);
    double *X = (double *)(wb + L.x_off);
    WS<float> ws{(float *)(wb + L.wd_off), (int *)(wb + L.wi_off), (int64_t)L.nblk * kWsDbl,
                 (int64_t)L.nblk * kWsInt};
    const SysDesc sd{2, dm.m32_off};
    const int rhs_cols = maxf + 1;
    auto back_solve = [&]() { run_back_solve<float, 2>(ctx, sd, e0, ne, M, ws, maxn, rhs_cols, s); };
    auto forward_solve = [&]() { run_forward_solve<float, 2>(ctx, sd, e0, ne, M, ws, maxn, rhs_cols, s); };
    const int tn = (rhs_cols + kTN - 1) / kTN;
    const dim3 elem_grid(64, ne);
    hipLaunchKernelGGL(k_to32, elem_grid, dim3(256), 0, s, dm, e0, (const double *)E, M);
    // FP32 LU of A with the forward substitution of [B | R_qu] carried along, then X_0
    int err = run_lu<float, 2>(ctx, sd, e0, ne, M, info, ws, true, maxn, maxn, maxn + maxf + 1, maxf + 1, 0, s);
    if (err) return err;
    back_solve();
    hipLaunchKernelGGL(k_xupdate<0>, elem_grid, dim3(256), 0, s, dm, e0, (const float *)M, X, E);
    const int tm_r = (maxn + kTM - 1) / kTM;
    for (int it = 0; it < refine; ++it) {
        // R = [B | R_qu] - A X in FP64 (into the FP32 right-hand columns), d = A^{-1} R, X += d
        hipLaunchKernelGGL(k_gemm64<0>, dim3(xcd_grid(ne, tm_r * tn)), dim3(256), 0, s, dm, e0, ne, tm_r, tn,
                           (const double *)E, (const double *)X, M, SK);
        forward_solve();
        back_solve();
        if (it + 1 < refine)
            hipLaunchKernelGGL(k_xupdate<1>, elem_grid, dim3(256), 0, s, dm, e0, (const float *)M, X, E);
        else
            hipLaunchKernelGGL(k_xupdate<2>, elem_grid, dim3(256), 0, s, dm, e0, (const float *)M, X, E);
    }
    // [S^K | -g^K] = [D | R_uh] - C X (FP64), stored as [S^K | g^K]
    const int tm_s = (maxf + kTM - 1) / kTM;
    hipLaunchKernelGGL(k_gemm64<1>, dim3(xcd_grid(ne, tm_s * tn)), dim3(256), 0, s, dm, e0, ne, tm_s, tn,
                       (const double *)E, (const double *)X, M, SK);
    return (int)hipGetLastError();
}

}  // namespace hdg
