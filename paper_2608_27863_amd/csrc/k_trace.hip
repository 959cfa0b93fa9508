// Trace-space kernels: assembly of the condensed system (eq. schur-trace),
// the block-sparse matvec, the one-level additive Schwarz preconditioner
// (eq. additive-schwarz), left-preconditioned GMRES, and the interior
// recovery (eq. local-elimination).  Every sum over element contributions is
// a gather in a fixed order: results are bit-reproducible, no atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "hdg_internal.h"

namespace hdg {
namespace {

typedef double v2d __attribute__((ext_vector_type(2)));


// ------------------------------------------------------------------ assembly
__global__ void __launch_bounds__(256) k_assemble_blocks(DevMesh dm, const double *__restrict__ SK,
                                                         double *__restrict__ S) {
    const int k = blockIdx.x;
    const int c0 = dm.blk_src_ptr[k], c1 = dm.blk_src_ptr[k + 1];
    const int e_first = dm.blk_src[3 * c0], a_first = dm.blk_src[3 * c0 + 1], b_first = dm.blk_src[3 * c0 + 2];
    const int *tf = dm.toff + 7 * e_first;
    const int bF = tf[a_first + 1] - tf[a_first], bG = tf[b_first + 1] - tf[b_first];
    double *out = S + dm.bsr_val_off[k];
    for (int t = threadIdx.x; t < bF * bG; t += blockDim.x) {
        const int ii = t % bF, jj = t / bF;
        double v = 0.0;
        for (int c = c0; c < c1; ++c) {
            const int e = dm.blk_src[3 * c], a = dm.blk_src[3 * c + 1], b = dm.blk_src[3 * c + 2];
            const int *to = dm.toff + 7 * e;
            const int fe = to[6];
            v += SK[dm.SK_off[e] + (int64_t)(to[b] + jj) * fe + to[a] + ii];
        }
        out[t] = v;
    }
    // the block's padding up to the next 128-byte line
    const int pad_end = (int)(dm.bsr_val_off[k + 1] - dm.bsr_val_off[k]);
    for (int t = bF * bG + threadIdx.x; t < pad_end; t += blockDim.x) out[t] = 0.0;
}

__global__ void __launch_bounds__(128) k_assemble_g(DevMesh dm, const double *__restrict__ SK, double *__restrict__ g) {
    const int F = blockIdx.x;
    const int bF = (int)(dm.face_off[F + 1] - dm.face_off[F]);
    const int s0 = dm.face_src_ptr[F], s1 = dm.face_src_ptr[F + 1];
    for (int i = threadIdx.x; i < bF; i += blockDim.x) {
        double v = 0.0;
        for (int s = s0; s < s1; ++s) {
            const int e = dm.face_src[2 * s], a = dm.face_src[2 * s + 1];
            const int *to = dm.toff + 7 * e;
            const int fe = to[6];
            v += SK[dm.SK_off[e] + (int64_t)fe * fe + to[a] + i];
        }
        g[dm.face_off[F] + i] = v;
    }
}

// -------------------------------------------------------------------- matvec
constexpr int kMaxRowBlocks = 16;
constexpr int kMvPiece = 4096;  // doubles of a block staged in LDS at a time (32 KB)

// One workgroup per face row F.  Each block (column-major bF x bG, starting on
// a 128-byte line, zero padding after it) is streamed through LDS in pieces of
// kMvPiece doubles, every thread with eight nontemporal 16-byte loads in flight
// over the piece's contiguous range, so every line is read once and whole.
// Thread (i, w) owns row i (i = tid mod bF, w = tid div bF < W = 256 div bF)
// and sums S[i][j] x[j] over its columns j = w mod W in increasing j; the W
// partial sums are added in order of w, so the result does not depend on
// timing.
__global__ void __launch_bounds__(256) k_matvec(DevMesh dm, const double *__restrict__ S,
                                                const double *__restrict__ x, double *__restrict__ y) {
    const int F = blockIdx.x;
    const int bF = (int)(dm.face_off[F + 1] - dm.face_off[F]);
    const int k0 = dm.bsr_row_ptr[F], nk = dm.bsr_row_ptr[F + 1] - k0;
    const int tid = threadIdx.x;
    __shared__ __attribute__((aligned(16))) double sp[kMvPiece];
    __shared__ double sx[kMaxRowBlocks * 125];
    __shared__ int sxo[kMaxRowBlocks + 1];
    __shared__ double sred[256];
    if (tid == 0) {
        int o = 0;
        for (int q = 0; q < nk; ++q) {
            sxo[q] = o;
            const int G = dm.bsr_col[k0 + q];
            o += (int)(dm.face_off[G + 1] - dm.face_off[G]);
        }
        sxo[nk] = o;
    }
    __syncthreads();
    for (int q = 0; q < nk; ++q) {
        const int G = dm.bsr_col[k0 + q];
        const int bG = sxo[q + 1] - sxo[q];
        for (int t = tid; t < bG; t += blockDim.x) sx[sxo[q] + t] = x[dm.face_off[G] + t];
    }
    const int W = 256 / bF;
    const int i = tid % bF, w = tid / bF;
    double acc = 0.0;
    for (int q = 0; q < nk; ++q) {
        const double *blk = S + dm.bsr_val_off[k0 + q];
        const double *xs = sx + sxo[q];
        const int bG = sxo[q + 1] - sxo[q], n = bF * bG;
        for (int p0 = 0; p0 < n; p0 += kMvPiece) {
            const int len = min(kMvPiece, n - p0);
            const int units = (len + 1) / 2;  // an odd block's last unit takes one zero of the padding
            v2d v[kMvPiece / 2 / 256];
#pragma unroll
            for (int r = 0; r < kMvPiece / 2 / 256; ++r) {
                const int u = tid + 256 * r;
                if (u < units) v[r] = __builtin_nontemporal_load((const v2d *)(blk + p0) + u);
            }
            __syncthreads();  // the previous piece has been read (and, first, sx is complete)
#pragma unroll
            for (int r = 0; r < kMvPiece / 2 / 256; ++r) {
                const int u = tid + 256 * r;
                if (u < units) *(v2d *)(sp + 2 * u) = v[r];
            }
            __syncthreads();
            if (w < W) {
                // columns j with j bF + i in [p0, p0 + len) and j = w mod W
                const int jlo = (p0 > i) ? (p0 - i + bF - 1) / bF : 0;
                const int last = p0 + len - 1 - i;
                const int jhi = last >= 0 ? last / bF : -1;
                int j = jlo + ((w - jlo % W) + W) % W;
                for (; j + 3 * W <= jhi; j += 4 * W) {
                    acc += sp[j * bF + i - p0] * xs[j];
                    acc += sp[(j + W) * bF + i - p0] * xs[j + W];
                    acc += sp[(j + 2 * W) * bF + i - p0] * xs[j + 2 * W];
                    acc += sp[(j + 3 * W) * bF + i - p0] * xs[j + 3 * W];
                }
                for (; j <= jhi; j += W) acc += sp[j * bF + i - p0] * xs[j];
            }
        }
    }
    sred[tid] = acc;
    __syncthreads();
    if (tid < bF) {
        double v = 0.0;
        for (int ww = 0; ww < W; ++ww) v += sred[ww * bF + tid];
        y[dm.face_off[F] + tid] = v;
    }
}

// ------------------------------------------------------------- Schwarz setup
// Systems [S_r' | I] (m rows, row-major, row stride e_ld(m, m) = 2m + 8), m = f
// rounded up to a multiple of 4; S_r' = [[S_r, 0], [0, I]] (decoupled padding
// unknowns).  k_asm_build writes the columns 0 .. m-1, one 32 x 32 tile per
// workgroup: read with consecutive lanes on consecutive rows (the BSR blocks are
// column-major), written through LDS with consecutive lanes on consecutive
// columns (the system is row-major); k_asm_identity writes the columns
// m .. 2m+7 (the identity, then zeros) with 16-byte nontemporal stores.
template <typename T>
__global__ void __launch_bounds__(256) k_asm_build(DevMesh dm, const double *__restrict__ S, T *__restrict__ sys) {
    const int e = blockIdx.z;
    const int *to = dm.toff + 7 * e;
    const int f = to[6], m = asm_pad(f);
    const int ld = (int)e_ld(m, m);
    const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
    if (r0 >= m || c0 >= m) return;  // uniform per block
    T *base = sys + dm.asmsys_off[e];
    __shared__ double tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = r0 + tx, c = c0 + ty + 8 * q;
        double v = 0.0;
        if (r < m && c < m) {
            if (r < f && c < f) {
                int a = 0, b = 0;
                while (r >= to[a + 1]) ++a;
                while (c >= to[b + 1]) ++b;
                const int k = dm.asm_blk[36 * e + 6 * a + b];
                const int bF = to[a + 1] - to[a];
                v = S[dm.bsr_val_off[k] + (r - to[a]) + (int64_t)(c - to[b]) * bF];
            } else {
                v = (r == c) ? 1.0 : 0.0;
            }
        }
        tile[tx][ty + 8 * q] = v;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int r = r0 + ty + 8 * q, c = c0 + tx;
        if (r < m && c < m) base[(int64_t)r * ld + c] = (T)tile[ty + 8 * q][tx];
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_asm_identity(DevMesh dm, T *__restrict__ sys) {
    constexpr int kVN = 16 / (int)sizeof(T);
    typedef T vq __attribute__((ext_vector_type(kVN)));
    const int e = blockIdx.y;
    const int f = dm.toff[7 * e + 6], m = asm_pad(f);
    const int64_t ld = e_ld(m, m);
    const int nv = (int)(ld - m) / kVN;  // 16-byte units of a row's right part (ld - m = m + 8)
    T *base = sys + dm.asmsys_off[e] + m;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < (int64_t)m * nv; t += (int64_t)gridDim.x * 256) {
        const int r = (int)(t / nv), u = (int)(t % nv);
        vq v;
#pragma unroll
        for (int i = 0; i < kVN; ++i) v[i] = (kVN * u + i == r) ? T(1) : T(0);
        __builtin_nontemporal_store(v, (vq *)(base + (int64_t)r * ld + kVN * u));
    }
}

// Sinv (column-major f x f) = the identity columns after the solve
template <typename T>
__global__ void __launch_bounds__(256) k_asm_extract(DevMesh dm, const T *__restrict__ sys, T *__restrict__ Sinv) {
    const int e = blockIdx.z;
    const int f = dm.toff[7 * e + 6], m = asm_pad(f);
    const int64_t ld = e_ld(m, m);
    const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 32;
    if (i0 >= f || j0 >= f) return;
    const T *base = sys + dm.asmsys_off[e];
    T *out = Sinv + dm.asm_off[e];
    __shared__ T tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int i = i0 + r, j = j0 + tx;
        tile[r][tx] = (i < f && j < f) ? base[(int64_t)i * ld + m + j] : T(0);
    }
    __syncthreads();
    for (int c = ty; c < 32; c += 8) {
        const int j = j0 + c, i = i0 + tx;
        if (i < f && j < f) out[(int64_t)j * f + i] = tile[tx][c];
    }
    if (blockIdx.x == 0 && blockIdx.y == 0) {  // the block's padding up to the next 128-byte line
        const int64_t pad_end = dm.asm_off[e + 1] - dm.asm_off[e];
        for (int64_t t = (int64_t)f * f + threadIdx.x; t < pad_end; t += blockDim.x) out[t] = T(0);
    }
}

// ------------------------------------------------------------- Schwarz apply
// zloc = S_r^{-1} y_r, y_r gathered from the element's six faces.  One
// workgroup per (element, 256 rows); the column-major inverse is streamed with
// consecutive lanes on consecutive rows, eight columns in flight per thread.
template <typename T>
__global__ void __launch_bounds__(256) k_asm_local(DevMesh dm, const T *__restrict__ Sinv, const double *__restrict__ r,
                                                   double *__restrict__ zloc) {
    const int e = blockIdx.x;
    const int *to = dm.toff + 7 * e;
    const int f = to[6];
    if ((int)blockIdx.y * 256 >= f) return;  // uniform per block
    __shared__ double sy[750];
    for (int lf = 0; lf < 6; ++lf) {
        const int F = dm.elem_face[6 * e + lf];
        const int len = to[lf + 1] - to[lf];
        for (int t = threadIdx.x; t < len; t += blockDim.x) sy[to[lf] + t] = r[dm.face_off[F] + t];
    }
    __syncthreads();
    const T *M = Sinv + dm.asm_off[e];
    const int i = blockIdx.y * 256 + threadIdx.x;
    if (i >= f) return;
    double acc = 0.0;
    int j = 0;
    for (; j + 7 < f; j += 8) {
        double a[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) a[q] = (double)M[(int64_t)(j + q) * f + i];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc += a[q] * sy[j + q];
    }
    for (; j < f; ++j) acc += (double)M[(int64_t)j * f + i] * sy[j];
    zloc[dm.tloc_off[e] + i] = acc;
}

// The same product with one workgroup per element, for inverses whose columns
// do not start on 128-byte lines (f <= 768).  The element's block (starting on a
// line, zero padding after it) streams through LDS in 32 KB pieces with
// nontemporal 16-byte loads, eight in flight per thread, so every line is read
// once and whole; each thread owns rows i, i + 256, i + 512 and sums over j in
// the same order as k_asm_local, so the two give identical results.
constexpr int kAsmRowsPerThread = 3;
constexpr int kAsmPieceBytes = 32768;

template <typename T>
__global__ void __launch_bounds__(256) k_asm_local_elem(DevMesh dm, const T *__restrict__ Sinv,
                                                        const double *__restrict__ r, double *__restrict__ zloc) {
    constexpr int kPiece = kAsmPieceBytes / (int)sizeof(T);  // entries per piece
    constexpr int kVN = 16 / (int)sizeof(T);                 // entries per 16-byte load
    constexpr int kLoads = kPiece / kVN / 256;                 // loads per thread and piece
    typedef T vq __attribute__((ext_vector_type(kVN)));
    const int e = blockIdx.x, tid = threadIdx.x;
    const int *to = dm.toff + 7 * e;
    const int f = to[6];
    __shared__ __attribute__((aligned(16))) T sp[kPiece];
    __shared__ double sy[kAsmRowsPerThread * 256];
    for (int lf = 0; lf < 6; ++lf) {
        const int F = dm.elem_face[6 * e + lf];
        const int len = to[lf + 1] - to[lf];
        for (int t = tid; t < len; t += blockDim.x) sy[to[lf] + t] = r[dm.face_off[F] + t];
    }
    const T *M = Sinv + dm.asm_off[e];
    const int64_t n = (int64_t)f * f;
    double acc[kAsmRowsPerThread] = {};
    for (int64_t p0 = 0; p0 < n; p0 += kPiece) {
        const int len = (int)min((int64_t)kPiece, n - p0);
        const int units = (len + kVN - 1) / kVN;  // the last unit may take zeros of the padding
        vq v[kLoads];
#pragma unroll
        for (int q = 0; q < kLoads; ++q) {
            const int u = tid + 256 * q;
            if (u < units) v[q] = __builtin_nontemporal_load((const vq *)(M + p0) + u);
        }
        __syncthreads();  // the previous piece has been read (and, first, sy is complete)
#pragma unroll
        for (int q = 0; q < kLoads; ++q) {
            const int u = tid + 256 * q;
            if (u < units) *(vq *)(sp + kVN * u) = v[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kAsmRowsPerThread; ++q) {
            const int i = tid + 256 * q;
            if (i >= f) continue;
            // columns j with j f + i in [p0, p0 + len)
            const int jlo = p0 > i ? (int)((p0 - i + f - 1) / f) : 0;
            const int64_t last = p0 + len - 1 - i;
            const int jhi = last >= 0 ? (int)(last / f) : -1;
            const T *col = sp + ((int64_t)jlo * f + i - p0);
            for (int j = jlo; j <= jhi; ++j, col += f) acc[q] += (double)*col * sy[j];
        }
    }
    double *z = zloc + dm.tloc_off[e];
#pragma unroll
    for (int q = 0; q < kAsmRowsPerThread; ++q)
        if (tid + 256 * q < f) z[tid + 256 * q] = acc[q];
}

__global__ void __launch_bounds__(128) k_asm_gather(DevMesh dm, const double *__restrict__ zloc, double *__restrict__ z) {
    const int F = blockIdx.x;
    const int bF = (int)(dm.face_off[F + 1] - dm.face_off[F]);
    const int s0 = dm.face_src_ptr[F], s1 = dm.face_src_ptr[F + 1];
    for (int i = threadIdx.x; i < bF; i += blockDim.x) {
        double v = 0.0;
        for (int s = s0; s < s1; ++s) {
            const int e = dm.face_src[2 * s], a = dm.face_src[2 * s + 1];
            v += zloc[dm.tloc_off[e] + dm.toff[7 * e + a] + i];
        }
        z[dm.face_off[F] + i] = v;
    }
}

// --------------------------------------------------------------------- GMRES
constexpr int kDotBlocks = 1024;  // four per CU
constexpr int kDotGroup = 8;      // vectors per pass over a block's slice of w

// partial[b * stride + v] = sum over block b's slice of V[v] . w   (v < nv).
// The vectors go kDotGroup at a time, so w is read once per group; each sum is
// reduced within a wave by shuffles and across the four waves through LDS, in
// a fixed order (deterministic).
__global__ void __launch_bounds__(256) k_dot_partial(const double *__restrict__ V, int nv, int64_t ldv,
                                                     const double *__restrict__ w, int64_t N,
                                                     double *__restrict__ partial, int stride) {
    __shared__ double red[4][kDotGroup];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t chunk = (N + gridDim.x - 1) / gridDim.x;
    const int64_t i0 = blockIdx.x * chunk, i1 = min(N, i0 + chunk);
    for (int v0 = 0; v0 < nv; v0 += kDotGroup) {
        const int ng = min(kDotGroup, nv - v0);
        double s[kDotGroup] = {};
        for (int64_t i = i0 + tid; i < i1; i += blockDim.x) {
            const double wi = w[i];
#pragma unroll
            for (int g = 0; g < kDotGroup; ++g)
                if (g < ng) s[g] += V[(int64_t)(v0 + g) * ldv + i] * wi;
        }
#pragma unroll
        for (int g = 0; g < kDotGroup; ++g) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) s[g] += __shfl_down(s[g], off, 64);
        }
        if (lane == 0) {
#pragma unroll
            for (int g = 0; g < kDotGroup; ++g) red[wave][g] = s[g];
        }
        __syncthreads();
        if (tid < ng) partial[(int64_t)blockIdx.x * stride + v0 + tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
        __syncthreads();
    }
}

// out[v] = (accumulate ? out[v] : 0) + sum_b partial[b * stride + v]; one block per v,
// fixed-shape tree (deterministic)
__global__ void __launch_bounds__(256) k_dot_final(const double *__restrict__ partial, int nblk, int stride, int nv,
                                                   double *__restrict__ out, int accumulate) {
    const int v = blockIdx.x;
    if (v >= nv) return;
    __shared__ double red[256];
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) s += partial[b * stride + v];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[v] = accumulate ? out[v] + red[0] : red[0];
}

// w -= sum_v coef[v] V[v]
__global__ void __launch_bounds__(256) k_sub_multi(const double *__restrict__ V, int nv, int64_t ldv,
                                                   const double *__restrict__ coef, double *__restrict__ w, int64_t N) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        double s = w[i];
        for (int v = 0; v < nv; ++v) s -= coef[v] * V[v * ldv + i];
        w[i] = s;
    }
}

// dst = src / *nrm  (0 if the norm is 0)
__global__ void __launch_bounds__(256) k_scale_inv(const double *__restrict__ src, const double *__restrict__ nrm_sq,
                                                   double *__restrict__ dst, int64_t N) {
    const double nr = sqrt(*nrm_sq);
    const double s = (nr > 0.0) ? 1.0 / nr : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i] * s;
}

// Start of the cycle: gam[0] = beta = ||r0||, hist[0] = beta.
__global__ void k_gmres_start(const double *__restrict__ nrm_sq, double *__restrict__ gam, double *__restrict__ hist, int m) {
    const double b = sqrt(*nrm_sq);
    for (int i = 0; i <= m; ++i) gam[i] = 0.0;
    gam[0] = b;
    hist[0] = b;
}

// Column j of H (length j+2, column-major ld m+1): fold in the norm, apply
// the previous rotations, form the new one, update gam and the history.
__global__ void k_givens(double *__restrict__ H, int m, int j, const double *__restrict__ nrm_sq,
                         double *__restrict__ cs, double *__restrict__ sn, double *__restrict__ gam,
                         double *__restrict__ hist) {
    double *h = H + (int64_t)j * (m + 1);
    h[j + 1] = sqrt(*nrm_sq);
    for (int i = 0; i < j; ++i) {
        const double t = cs[i] * h[i] + sn[i] * h[i + 1];
        h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
        h[i] = t;
    }
    const double a = h[j], b = h[j + 1];
    const double den = hypot(a, b);
    double c = 1.0, s = 0.0;
    if (den > 0.0) { c = a / den; s = b / den; }
    cs[j] = c;
    sn[j] = s;
    h[j] = den;
    h[j + 1] = 0.0;
    gam[j + 1] = -s * gam[j];
    gam[j] = c * gam[j];
    hist[j + 1] = fabs(gam[j + 1]);
}

// y = R^{-1} gam (upper triangular m x m part of H); skips zero pivots
__global__ void k_upper_solve(const double *__restrict__ H, int m, const double *__restrict__ gam, double *__restrict__ y) {
    for (int i = m - 1; i >= 0; --i) {
        double s = gam[i];
        for (int k = i + 1; k < m; ++k) s -= H[(int64_t)k * (m + 1) + i] * y[k];
        const double d = H[(int64_t)i * (m + 1) + i];
        y[i] = (d != 0.0) ? s / d : 0.0;
    }
}

// x = x0 + sum_v y[v] V[v]  (x0 = NULL: 0; x may alias x0)
__global__ void __launch_bounds__(256) k_combine(const double *__restrict__ V, int nv, int64_t ldv,
                                                 const double *__restrict__ y, const double *x0, double *x,
                                                 int64_t N) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        double s = x0 ? x0[i] : 0.0;
        for (int v = 0; v < nv; ++v) s += y[v] * V[v * ldv + i];
        x[i] = s;
    }
}

// t = g - t  (the initial residual g - S x0, with S x0 already in t)
__global__ void __launch_bounds__(256) k_rsub(const double *__restrict__ g, double *__restrict__ t, int64_t N) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        t[i] = g[i] - t[i];
}

__global__ void __launch_bounds__(256) k_copy(const double *__restrict__ src, double *__restrict__ dst, int64_t N) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// ------------------------------------------------------ reduced basis (eq. rb-min)
// Column j of the QR factorisation of Z by classical Gram-Schmidt applied
// twice: after the two projections, q (in Qz[j]) has norm^2 *nrm_sq and the
// column before them *z_sq.  A column whose part orthogonal to the previous
// ones is below kRbDrop of its norm is dependent on them: it gets R_jj = 0 and
// q = 0, and its coefficient is then 0 (the kept columns span the same space).
constexpr double kRbDrop = 1e-12;
__global__ void k_rb_diag(const double *__restrict__ nrm_sq, const double *__restrict__ z_sq, double *__restrict__ Rjj) {
    const double nr = sqrt(*nrm_sq), nz = sqrt(*z_sq);
    *Rjj = (nr > kRbDrop * nz && nr > 0.0) ? nr : 0.0;
}
// dst = src / *d (0 if *d is 0)
__global__ void __launch_bounds__(256) k_scale_by(const double *__restrict__ src, const double *__restrict__ d,
                                                  double *__restrict__ dst, int64_t N) {
    const double s = (*d != 0.0) ? 1.0 / *d : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i] * s;
}

// ------------------------------------------------------------ Newton update
// W += alpha dW (eq. newton-update): Q, U from the packed interior increment
// dQU ([e][20][node]: 15 gradient fields, then 5 conserved), Uhat from dUhat.
__global__ void __launch_bounds__(256) k_state_update(DevMesh dm, double alpha, const double *__restrict__ dQU,
                                                      const double *__restrict__ dUhat, double *__restrict__ Q,
                                                      double *__restrict__ U, double *__restrict__ Uhat) {
    const int e = blockIdx.x;
    if (e < dm.n_elem) {
        const int p = dm.elem_p[e], Np = (p + 1) * (p + 1) * (p + 1);
        const int64_t o = dm.node_off[e];
        const double *d = dQU + 20 * o;
        for (int i = threadIdx.x; i < 15 * Np; i += blockDim.x) Q[15 * o + i] += alpha * d[i];
        for (int i = threadIdx.x; i < 5 * Np; i += blockDim.x) U[5 * o + i] += alpha * d[15 * Np + i];
    }
    // the trace: faces spread over the same blocks
    const int64_t N = dm.face_off[dm.n_face];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        Uhat[i] += alpha * dUhat[i];
}

// out = sum_k coef[k] v_k over n values (k < 8): the DIRK combinations of
// eqs. dirk-stage and dirk-update
struct LinComb {
    const double *v[8];
    double c[8];
    int k;
};
__global__ void __launch_bounds__(256) k_lincomb(LinComb lc, double *__restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < lc.k; ++k) s += lc.c[k] * lc.v[k][i];
        out[i] = s;
    }
}

// Nonlinear residual norm (eq. nonlinear-residual), from element systems just
// written by the residual kernels: per element, the sums of squares of R_q and
// R_u into part[2 e], [2 e + 1], and the element-side trace residual R_uh^K
// copied to ruh_loc (element-local trace order) for the face assembly.
__global__ void __launch_bounds__(256) k_resid_elem(DevMesh dm, int e0, const double *__restrict__ Ebase,
                                                    double *__restrict__ part, double *__restrict__ ruh_loc) {
    const int e = e0 + blockIdx.x;
    const int p = dm.elem_p[e], Np = (p + 1) * (p + 1) * (p + 1), n = 20 * Np;
    const int f = dm.toff[7 * e + 6];
    const int64_t ld = e_ld(n, f);
    const double *E = Ebase + (dm.E_off[e] - dm.E_off[e0]);
    __shared__ double red[2][256];
    double sq = 0.0, su = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double r = E[(int64_t)i * ld + n + f];
        if (i < 15 * Np) sq += r * r;
        else su += r * r;
    }
    for (int a = threadIdx.x; a < f; a += blockDim.x) ruh_loc[dm.tloc_off[e] + a] = E[(int64_t)(n + a) * ld + n + f];
    red[0][threadIdx.x] = sq;
    red[1][threadIdx.x] = su;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * e] = red[0][0];
        part[2 * e + 1] = red[1][0];
    }
}

// Per face: the assembled trace residual R_uh[F] = sum over the face's
// elements of R_uh^K (fixed order), its sum of squares into fpart[F].
__global__ void __launch_bounds__(128) k_resid_face(DevMesh dm, const double *__restrict__ ruh_loc,
                                                    double *__restrict__ fpart) {
    const int F = blockIdx.x;
    const int bF = (int)(dm.face_off[F + 1] - dm.face_off[F]);
    const int s0 = dm.face_src_ptr[F], s1 = dm.face_src_ptr[F + 1];
    __shared__ double red[128];
    double acc = 0.0;
    for (int i = threadIdx.x; i < bF; i += blockDim.x) {
        double v = 0.0;
        for (int s = s0; s < s1; ++s) {
            const int e = dm.face_src[2 * s], a = dm.face_src[2 * s + 1];
            v += ruh_loc[dm.tloc_off[e] + dm.toff[7 * e + a] + i];
        }
        acc += v * v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 64; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) fpart[F] = red[0];
}

// out[0..2] = ||R_q||, ||R_u||, ||R_uh|| from the per-element and per-face
// partial sums (one block, fixed-shape tree: deterministic)
__global__ void __launch_bounds__(256) k_resid_final(const double *__restrict__ part, int ne,
                                                     const double *__restrict__ fpart, int nf, double *__restrict__ out) {
    __shared__ double red[3][256];
    double a = 0.0, b = 0.0, c = 0.0;
    for (int e = threadIdx.x; e < ne; e += blockDim.x) {
        a += part[2 * e];
        b += part[2 * e + 1];
    }
    for (int F = threadIdx.x; F < nf; F += blockDim.x) c += fpart[F];
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    red[2][threadIdx.x] = c;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h)
            for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int q = 0; q < 3; ++q) out[q] = sqrt(red[q][0]);
}

__global__ void k_zero_flag(int *flag) { flag[0] = 0; }

// Admissibility of W + alpha dW at the nodes: flag[0] = 1 if any node would
// have non-positive density or pressure (or a non-finite value), else
// untouched (k_zero_flag clears it first).
__global__ void __launch_bounds__(256) k_admissible(DevMesh dm, double alpha, double gamma, const double *__restrict__ U,
                                                    const double *__restrict__ dQU, int *__restrict__ flag) {
    const int e = blockIdx.x;
    const int p = dm.elem_p[e], Np = (p + 1) * (p + 1) * (p + 1);
    const int64_t o = dm.node_off[e];
    const double *u = U + 5 * o;
    const double *d = dQU + 20 * o + 15 * Np;
    bool bad = false;
    for (int i = threadIdx.x; i < Np; i += blockDim.x) {
        double w[5];
        for (int c = 0; c < 5; ++c) w[c] = u[c * Np + i] + alpha * d[c * Np + i];
        const double rho = w[0];
        const double ke = 0.5 * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]) / rho;
        const double pr = (gamma - 1.0) * (w[4] - ke);
        if (!(rho > 0.0) || !(pr > 0.0) || !isfinite(pr)) bad = true;
    }
    if (bad) flag[0] = 1;
}

// ------------------------------------------------------------------ recovery
// y_i = E[i][n+f] + sum_j E[i][n+j] dUh^K_j for i < n, then (FP64) back
// substitution with the upper triangle of E's first n columns; dQU = -x.  One
// 1024-thread workgroup per element.  Every row product is one wave reading
// the row's entries with consecutive lanes (coalesced), four rows in flight
// per wave, then a shuffle reduction.  The back substitution goes by 64-row
// blocks: the diagonal block by wave 0 in LDS, then the rows above update
// with the block's solution.
constexpr int kRB = 64, kRT = 1024, kRW = kRT / 64, kRQ = 4;  // kRQ rows in flight per wave

// Y = [Y_B | y_r] is read from the chunk's element systems (columns n.., row
// stride e_ld) or, with Xbase, from the retained X (columns 0.., stride x_ld).
__global__ void __launch_bounds__(kRT) k_recover(DevMesh dm, int e0, int backsub, const double *__restrict__ Ebase,
                                                 const double *__restrict__ Xbase, const double *__restrict__ dUhat,
                                                 double *__restrict__ dQU) {
    const int e = e0 + blockIdx.x;
    const int p = dm.elem_p[e], Np = (p + 1) * (p + 1) * (p + 1), n = 20 * Np;
    const int *to = dm.toff + 7 * e;
    const int f = to[6];
    const int64_t ld = e_ld(n, f);
    const double *E = Xbase ? nullptr : Ebase + (dm.E_off[e] - dm.E_off[e0]);
    const double *Y = Xbase ? Xbase + dm.x_off[e] : E + n;
    const int64_t ldy = Xbase ? x_ld(f) : ld;
    __shared__ double sd[750];
    __shared__ double sy[2500];
    __shared__ double sU[kRB][kRB + 1];
    for (int lf = 0; lf < 6; ++lf) {
        const int F = dm.elem_face[6 * e + lf];
        const int len = to[lf + 1] - to[lf];
        for (int t = threadIdx.x; t < len; t += blockDim.x) sd[to[lf] + t] = dUhat[dm.face_off[F] + t];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    auto wave_sum = [&](double v) {
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        return v;
    };
    // y = Y_r + Y_B dUh, kRQ rows per wave at a time
    for (int i = kRQ * wave; i < n; i += kRQ * kRW) {
        double acc[kRQ];
#pragma unroll
        for (int q = 0; q < kRQ; ++q) acc[q] = 0.0;
        // four column strides' loads in flight per lane; every acc[q] still adds its
        // terms in increasing j
        for (int j0 = lane; j0 < f; j0 += 4 * 64) {
            double yv[4][kRQ];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int q = 0; q < kRQ; ++q) {
                    const int j = j0 + 64 * u;
                    yv[u][q] = (j < f && i + q < n) ? Y[(int64_t)(i + q) * ldy + j] : 0.0;
                }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = j0 + 64 * u;
                if (j < f) {
                    const double dj = sd[j];
#pragma unroll
                    for (int q = 0; q < kRQ; ++q)
                        if (i + q < n) acc[q] += yv[u][q] * dj;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < kRQ; ++q) {
            const double v = wave_sum(acc[q]);
            if (lane == 0 && i + q < n) sy[i + q] = v + Y[(int64_t)(i + q) * ldy + f];
        }
    }
    __syncthreads();
    if (backsub) {
        // left-looking by 64-row blocks from the bottom: a block's rows first take
        // the solved part, y[r] -= U[r][i1:n] x[i1:n] (one dot product per row,
        // kRQ rows per wave), then wave 0 solves the diagonal block
        for (int i1 = n; i1 > 0; i1 -= kRB) {
            const int i0 = max(0, i1 - kRB), nb = i1 - i0;
            for (int r = i0 + kRQ * wave; r < i1; r += kRQ * kRW) {
                double acc[kRQ];
#pragma unroll
                for (int q = 0; q < kRQ; ++q) acc[q] = 0.0;
                for (int c0 = i1 + lane; c0 < n; c0 += 4 * 64) {
                    double uv[4][kRQ];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int q = 0; q < kRQ; ++q) {
                            const int c = c0 + 64 * u;
                            uv[u][q] = (c < n && r + q < i1) ? E[(int64_t)(r + q) * ld + c] : 0.0;
                        }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int c = c0 + 64 * u;
                        if (c < n) {
                            const double xc = sy[c];
#pragma unroll
                            for (int q = 0; q < kRQ; ++q)
                                if (r + q < i1) acc[q] += uv[u][q] * xc;
                        }
                    }
                }
#pragma unroll
                for (int q = 0; q < kRQ; ++q) {
                    const double t = wave_sum(acc[q]);
                    if (lane == 0 && r + q < i1) sy[r + q] -= t;
                }
            }
            for (int t = threadIdx.x; t < kRB * kRB; t += blockDim.x) {
                const int r = t / kRB, c = t % kRB;
                sU[r][c] = (r < nb && c < nb) ? E[(int64_t)(i0 + r) * ld + i0 + c] : 0.0;
            }
            __syncthreads();
            if (wave == 0) {
                // diagonal block: lanes hold rows i0 + lane
                double yl = (lane < nb) ? sy[i0 + lane] : 0.0;
                for (int c = nb - 1; c >= 0; --c) {
                    const double xc = __shfl(yl, c) / sU[c][c];
                    if (lane == c) yl = xc;
                    else if (lane < c) yl -= sU[lane][c] * xc;
                }
                if (lane < nb) sy[i0 + lane] = yl;
            }
            __syncthreads();
        }
    }
    double *out = dQU + 20 * dm.node_off[e];
    for (int i = threadIdx.x; i < n; i += blockDim.x) out[i] = -sy[i];
}

// X of one element (rows 0..n-1, columns n..n+f of its condensed system) to
// the retained store, kStoreXRows rows per workgroup, padding columns zeroed.
constexpr int kStoreXRows = 16;
__global__ void __launch_bounds__(256) k_store_x(DevMesh dm, int e0, const double *__restrict__ Ebase,
                                                 double *__restrict__ X) {
    const int e = e0 + blockIdx.y;
    const int p = dm.elem_p[e], n = 20 * (p + 1) * (p + 1) * (p + 1);
    const int f = dm.toff[7 * e + 6];
    const int r0 = blockIdx.x * kStoreXRows;
    if (r0 >= n) return;
    const int64_t ld = e_ld(n, f), xl = x_ld(f);
    const double *E = Ebase + (dm.E_off[e] - dm.E_off[e0]) + n;
    double *Xe = X + dm.x_off[e];
    const int rows = min(kStoreXRows, n - r0);
    for (int t = threadIdx.x; t < rows * xl; t += blockDim.x) {
        const int r = r0 + t / (int)xl, c = t % (int)xl;
        Xe[(int64_t)r * xl + c] = c <= f ? E[(int64_t)r * ld + c] : 0.0;
    }
}

inline int grid_for(int64_t n, int threads = 256, int cap = 2048) {
    int64_t g = (n + threads - 1) / threads;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

}  // namespace

int launch_assemble(const hdg_ctx *ctx, const double *SK, double *S, double *g, hipStream_t s) {
    const DevMesh &dm = ctx->dm;
    const int nnzb = (int)ctx->bsr_col.size();
    hipLaunchKernelGGL(k_assemble_blocks, dim3(nnzb), dim3(256), 0, s, dm, SK, S);
    hipLaunchKernelGGL(k_assemble_g, dim3(ctx->n_face), dim3(128), 0, s, dm, SK, g);
    return (int)hipGetLastError();
}

int launch_matvec(const hdg_ctx *ctx, const double *S, const double *x, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_matvec, dim3(ctx->n_face), dim3(256), 0, s, ctx->dm, S, x, y);
    return (int)hipGetLastError();
}

size_t asm_setup_work_bytes(const hdg_ctx *ctx, int prec) {
    const size_t es = (prec == HDG_FP64) ? sizeof(double) : sizeof(float);
    size_t sys = es * (size_t)ctx->asmsys_off[ctx->n_elem];
    return (sys + 255) / 256 * 256 + (schwarz_ws_bytes(ctx, prec) + 255) / 256 * 256;
}

int launch_asm_setup(const hdg_ctx *ctx, int prec, const double *S, void *Sinv, int *info, void *work,
                     hipStream_t s) {
    const DevMesh &dm = ctx->dm;
    void *sys = work;
    const size_t es = (prec == HDG_FP64) ? sizeof(double) : sizeof(float);
    size_t sys_bytes = (es * (size_t)ctx->asmsys_off[ctx->n_elem] + 255) / 256 * 256;
    void *iwork = (void *)((char *)work + sys_bytes);
    // FP64 inverses for FP64 storage; FP32 storage is inverted in FP32 (FP32 matrix cores)
    const int mmax = asm_pad(ctx->max_f);
    const dim3 bgrid((mmax + 31) / 32, (mmax + 31) / 32, ctx->n_elem);
    const dim3 igrid(32, ctx->n_elem);
    if (prec == HDG_FP64) {
        hipLaunchKernelGGL(k_asm_build<double>, bgrid, dim3(256), 0, s, dm, S, (double *)sys);
        hipLaunchKernelGGL(k_asm_identity<double>, igrid, dim3(256), 0, s, dm, (double *)sys);
    } else {
        hipLaunchKernelGGL(k_asm_build<float>, bgrid, dim3(256), 0, s, dm, S, (float *)sys);
        hipLaunchKernelGGL(k_asm_identity<float>, igrid, dim3(256), 0, s, dm, (float *)sys);
    }
    int err = run_asm_inversion(ctx, prec, sys, info, iwork, s);
    if (err) return err;
    const int maxf = ctx->max_f;
    dim3 grid((maxf + 31) / 32, (maxf + 31) / 32, ctx->n_elem);
    if (prec == HDG_FP64)
        hipLaunchKernelGGL(k_asm_extract<double>, grid, dim3(256), 0, s, dm, (const double *)sys, (double *)Sinv);
    else
        hipLaunchKernelGGL(k_asm_extract<float>, grid, dim3(256), 0, s, dm, (const float *)sys, (float *)Sinv);
    return (int)hipGetLastError();
}

size_t asm_apply_work_bytes(const hdg_ctx *ctx) {
    return (sizeof(double) * (size_t)ctx->tloc_off[ctx->n_elem] + 255) / 256 * 256;
}

int launch_asm_apply(const hdg_ctx *ctx, int prec, const void *Sinv, const double *r, double *z, void *work,
                     hipStream_t s) {
    const DevMesh &dm = ctx->dm;
    double *zloc = (double *)work;
    const dim3 grid(ctx->n_elem, (ctx->max_f + 255) / 256);
    const bool aligned = prec == HDG_FP64 ? ctx->asm_cols_aligned64 : ctx->asm_cols_aligned32;
    const bool per_elem = !aligned && ctx->max_f <= kAsmRowsPerThread * 256;
    if (prec == HDG_FP64) {
        if (per_elem)
            hipLaunchKernelGGL(k_asm_local_elem<double>, dim3(ctx->n_elem), dim3(256), 0, s, dm, (const double *)Sinv, r,
                               zloc);
        else
            hipLaunchKernelGGL(k_asm_local<double>, grid, dim3(256), 0, s, dm, (const double *)Sinv, r, zloc);
    } else {
        if (per_elem)
            hipLaunchKernelGGL(k_asm_local_elem<float>, dim3(ctx->n_elem), dim3(256), 0, s, dm, (const float *)Sinv, r,
                               zloc);
        else
            hipLaunchKernelGGL(k_asm_local<float>, grid, dim3(256), 0, s, dm, (const float *)Sinv, r, zloc);
    }
    hipLaunchKernelGGL(k_asm_gather, dim3(ctx->n_face), dim3(128), 0, s, dm, (const double *)zloc, z);
    return (int)hipGetLastError();
}

// Workspace of hdg_asm_block_apply_noalloc: the element-local corrections
// zloc (sum of f_e doubles) in a library-owned array, one copy per device.
// Host code never passes `scratch` itself to a kernel (on the host the name
// is only a stand-in): it passes the device address recorded per device by
// asm_scratch_init.
static __device__ __align__(256) double scratch[kAsmScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

int asm_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[device]) return 0;
    double *ptr = nullptr;
    const hipError_t err = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (err != hipSuccess || !ptr) return err != hipSuccess ? (int)err : (int)hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
    return 0;
}

int launch_asm_apply_noalloc(const hdg_ctx *ctx, int prec, const void *Sinv, const double *r, double *z,
                             hipStream_t s) {
    double *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mutex);
        if (ctx->device >= 0 && ctx->device < kMaxDevices) ptr = g_scratch_ptr[ctx->device];
    }
    if (!ptr) return (int)hipErrorInvalidSymbol;
    return launch_asm_apply(ctx, prec, Sinv, r, z, ptr, s);
}

// GMRES workspace (doubles): V[(m+1) N] | w[N] | t[N] | zloc | H[(m+1) m] | cs[m] | sn[m] | gam[m+1] |
//                            hcol[m+1] | y[m] | partial[kDotBlocks (m+2)] | scal[8]
static size_t gmres_layout(const hdg_ctx *ctx, int m, size_t *off) {
    const size_t N = (size_t)ctx->face_off[ctx->n_face];
    const size_t nz = (size_t)ctx->tloc_off[ctx->n_elem];
    size_t o = 0;
    auto take = [&](size_t n) { size_t at = o; o += (n + 31) / 32 * 32; return at; };
    off[0] = take((m + 1) * N);
    off[1] = take(N);
    off[2] = take(N);
    off[3] = take(nz);
    off[4] = take((size_t)(m + 1) * m);
    off[5] = take(m);
    off[6] = take(m);
    off[7] = take(m + 1);
    off[8] = take(m + 1);
    off[9] = take(m);
    off[10] = take((size_t)kDotBlocks * (m + 2));
    off[11] = take(8);
    return o * sizeof(double);
}

size_t gmres_work_bytes(const hdg_ctx *ctx, int m) {
    size_t off[12];
    return gmres_layout(ctx, m, off);
}

int launch_gmres(const hdg_ctx *ctx, int prec, const double *S, const void *Sinv, const double *g, const double *x0,
                 int m, double *x, double *hist, void *work, hipStream_t s) {
    size_t off[12];
    gmres_layout(ctx, m, off);
    double *W = (double *)work;
    double *V = W + off[0], *w = W + off[1], *t = W + off[2], *zloc = W + off[3], *H = W + off[4];
    double *cs = W + off[5], *sn = W + off[6], *gam = W + off[7], *hcol = W + off[8], *y = W + off[9];
    double *partial = W + off[10], *scal = W + off[11];
    const int64_t N = ctx->face_off[ctx->n_face];
    const int stride = m + 2;
    const int gN = grid_for(N);
    int err;
    // r0 = M^{-1} (g - S x0), beta = ||r0||, v0 = r0 / beta
    if (x0) {
        if ((err = launch_matvec(ctx, S, x0, t, s))) return err;
        hipLaunchKernelGGL(k_rsub, dim3(gN), dim3(256), 0, s, g, t, N);
        if ((err = launch_asm_apply(ctx, prec, Sinv, t, w, zloc, s))) return err;
    } else {
        if ((err = launch_asm_apply(ctx, prec, Sinv, g, w, zloc, s))) return err;
    }
    hipLaunchKernelGGL(k_dot_partial, dim3(kDotBlocks), dim3(256), 0, s, (const double *)w, 1, (int64_t)0,
                       (const double *)w, N, partial, stride);
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, s, (const double *)partial, kDotBlocks, stride, 1, scal, 0);
    hipLaunchKernelGGL(k_gmres_start, dim3(1), dim3(1), 0, s, (const double *)scal, gam, hist, m);
    hipLaunchKernelGGL(k_scale_inv, dim3(gN), dim3(256), 0, s, (const double *)w, (const double *)scal, V, N);
    for (int j = 0; j < m; ++j) {
        double *vj = V + (int64_t)j * N;
        if ((err = launch_matvec(ctx, S, vj, t, s))) return err;
        if ((err = launch_asm_apply(ctx, prec, Sinv, t, w, zloc, s))) return err;
        double *hj = H + (int64_t)j * (m + 1);
        // classical Gram-Schmidt, applied twice
        for (int pass = 0; pass < 2; ++pass) {
            hipLaunchKernelGGL(k_dot_partial, dim3(kDotBlocks), dim3(256), 0, s, (const double *)V, j + 1, N,
                               (const double *)w, N, partial, stride);
            hipLaunchKernelGGL(k_dot_final, dim3(j + 1), dim3(256), 0, s, (const double *)partial,
                               kDotBlocks, stride, j + 1, pass == 0 ? hj : hcol, 0);
            hipLaunchKernelGGL(k_sub_multi, dim3(gN), dim3(256), 0, s, (const double *)V, j + 1, N,
                               (const double *)(pass == 0 ? hj : hcol), w, N);
            if (pass == 1)
                hipLaunchKernelGGL(k_dot_final, dim3(j + 1), dim3(256), 0, s, (const double *)partial,
                                   kDotBlocks, stride, j + 1, hj, 1);
        }
        hipLaunchKernelGGL(k_dot_partial, dim3(kDotBlocks), dim3(256), 0, s, (const double *)w, 1, (int64_t)0,
                           (const double *)w, N, partial, stride);
        hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, s, (const double *)partial, kDotBlocks, stride, 1, scal, 0);
        hipLaunchKernelGGL(k_scale_inv, dim3(gN), dim3(256), 0, s, (const double *)w, (const double *)scal,
                           V + (int64_t)(j + 1) * N, N);
        hipLaunchKernelGGL(k_givens, dim3(1), dim3(1), 0, s, H, m, j, (const double *)scal, cs, sn, gam, hist);
    }
    hipLaunchKernelGGL(k_upper_solve, dim3(1), dim3(1), 0, s, (const double *)H, m, (const double *)gam, y);
    hipLaunchKernelGGL(k_combine, dim3(gN), dim3(256), 0, s, (const double *)V, m, N, (const double *)y, x0, x, N);
    return (int)hipGetLastError();
}

// Reduced-basis guess workspace (doubles): Qz[nb N] | R[(nb+1) nb] | qg[nb] | c[nb] |
//                                         partial[kDotBlocks (nb+2)] | scal[8]
static size_t rb_layout(const hdg_ctx *ctx, int nb, size_t *off) {
    const size_t N = (size_t)ctx->face_off[ctx->n_face];
    size_t o = 0;
    auto take = [&](size_t n) { size_t at = o; o += (n + 31) / 32 * 32; return at; };
    off[0] = take((size_t)nb * N);
    off[1] = take((size_t)(nb + 1) * nb);
    off[2] = take(nb);
    off[3] = take(nb);
    off[4] = take((size_t)kDotBlocks * (nb + 2));
    off[5] = take(8);
    return o * sizeof(double);
}

size_t rb_work_bytes(const hdg_ctx *ctx, int nb_max) {
    size_t off[6];
    return rb_layout(ctx, nb_max, off);
}

// x0 = W c, c = argmin ||g - Z c||_2 over the `nb` stored columns
// (eq. rb-min): CGS2 QR of Z, c = R^{-1} Q^T g (dependent columns get c = 0).
int launch_rb_guess(const hdg_ctx *ctx, int nb, const double *Wb, const double *Zb, const double *g, double *x0,
                    void *work, hipStream_t s) {
    const int64_t N = ctx->face_off[ctx->n_face];
    const int gN = grid_for(N);
    if (nb == 0) {
        hipLaunchKernelGGL(k_combine, dim3(gN), dim3(256), 0, s, Wb, 0, N, (const double *)nullptr,
                           (const double *)nullptr, x0, N);
        return (int)hipGetLastError();
    }
    size_t off[6];
    rb_layout(ctx, nb, off);
    double *Wk = (double *)work;
    double *Qz = Wk + off[0], *R = Wk + off[1], *qg = Wk + off[2], *c = Wk + off[3];
    double *partial = Wk + off[4], *scal = Wk + off[5];
    const int ldr = nb + 1, stride = nb + 2;
    for (int j = 0; j < nb; ++j) {
        double *q = Qz + (int64_t)j * N;
        double *rj = R + (int64_t)j * ldr;
        hipLaunchKernelGGL(k_copy, dim3(gN), dim3(256), 0, s, Zb + (int64_t)j * N, q, N);
        // ||z_j||^2 -> scal[1]
        hipLaunchKernelGGL(k_dot_partial, dim3(kDotBlocks), dim3(256), 0, s, (const double *)q, 1, (int64_t)0,
                           (const double *)q, N, partial, stride);
        hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, s, (const double *)partial, kDotBlocks, stride, 1,
                           scal + 1, 0);
        if (j > 0) {
            for (int pass = 0; pass < 2; ++pass) {
                hipLaunchKernelGGL(k_dot_partial, dim3(kDotBlocks), dim3(256), 0, s, (const double *)Qz, j, N,
                                   (const double *)q, N, partial, stride);
                // pass 0 writes R[0..j-1, j]; pass 1 its correction (scal+2..), then adds it
                hipLaunchKernelGGL(k_dot_final, dim3(j), dim3(256), 0, s, (const double *)partial, kDotBlocks, stride,
                                   j, pass == 0 ? rj : c, 0);
                hipLaunchKernelGGL(k_sub_multi, dim3(gN), dim3(256), 0, s, (const double *)Qz, j, N,
                                   (const double *)(pass == 0 ? rj : c), q, N);
                if (pass == 1)
                    hipLaunchKernelGGL(k_dot_final, dim3(j), dim3(256), 0, s, (const double *)partial, kDotBlocks,
                                       stride, j, rj, 1);
            }
        }
        hipLaunchKernelGGL(k_dot_partial, dim3(kDotBlocks), dim3(256), 0, s, (const double *)q, 1, (int64_t)0,
                           (const double *)q, N, partial, stride);
        hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, s, (const double *)partial, kDotBlocks, stride, 1,
                           scal, 0);
        hipLaunchKernelGGL(k_rb_diag, dim3(1), dim3(1), 0, s, (const double *)scal, (const double *)(scal + 1), rj + j);
        hipLaunchKernelGGL(k_scale_by, dim3(gN), dim3(256), 0, s, (const double *)q, (const double *)(rj + j), q, N);
    }
    // qg = Q^T g, c = R^{-1} qg, x0 = W c
    hipLaunchKernelGGL(k_dot_partial, dim3(kDotBlocks), dim3(256), 0, s, (const double *)Qz, nb, N, g, N, partial,
                       stride);
    hipLaunchKernelGGL(k_dot_final, dim3(nb), dim3(256), 0, s, (const double *)partial, kDotBlocks, stride, nb, qg, 0);
    hipLaunchKernelGGL(k_upper_solve, dim3(1), dim3(1), 0, s, (const double *)R, nb, (const double *)qg, c);
    hipLaunchKernelGGL(k_combine, dim3(gN), dim3(256), 0, s, Wb, nb, N, (const double *)c, (const double *)nullptr,
                       x0, N);
    return (int)hipGetLastError();
}

// W[:, slot] = w_new, Z[:, slot] = S w_new
int launch_rb_insert(const hdg_ctx *ctx, const double *S, const double *w_new, int slot, double *Wb, double *Zb,
                     hipStream_t s) {
    const int64_t N = ctx->face_off[ctx->n_face];
    hipLaunchKernelGGL(k_copy, dim3(grid_for(N)), dim3(256), 0, s, w_new, Wb + (int64_t)slot * N, N);
    return launch_matvec(ctx, S, w_new, Zb + (int64_t)slot * N, s);
}

int launch_state_update(const hdg_ctx *ctx, double alpha, const double *dQU, const double *dUhat, double *Q,
                        double *U, double *Uhat, hipStream_t s) {
    hipLaunchKernelGGL(k_state_update, dim3(ctx->n_elem), dim3(256), 0, s, ctx->dm, alpha, dQU, dUhat, Q, U, Uhat);
    return (int)hipGetLastError();
}

int launch_lincomb(int k, const double *const *v, const double *c, double *out, int64_t n, hipStream_t s) {
    LinComb lc{};
    lc.k = k;
    for (int i = 0; i < k; ++i) {
        lc.v[i] = v[i];
        lc.c[i] = c[i];
    }
    hipLaunchKernelGGL(k_lincomb, dim3(grid_for(n)), dim3(256), 0, s, lc, out, n);
    return (int)hipGetLastError();
}

size_t resid_work_bytes(const hdg_ctx *ctx) {
    return sizeof(double) * ((size_t)2 * ctx->n_elem + (size_t)ctx->tloc_off[ctx->n_elem] + (size_t)ctx->n_face) + 256;
}

int launch_resid_elem(const hdg_ctx *ctx, int e0, int ne, const double *E, void *work, hipStream_t s) {
    double *part = (double *)work;
    double *ruh = part + 2 * (size_t)ctx->n_elem;
    hipLaunchKernelGGL(k_resid_elem, dim3(ne), dim3(256), 0, s, ctx->dm, e0, E, part, ruh);
    return (int)hipGetLastError();
}

int launch_resid_norm(const hdg_ctx *ctx, void *work, double *out, hipStream_t s) {
    double *part = (double *)work;
    double *ruh = part + 2 * (size_t)ctx->n_elem;
    double *fpart = ruh + (size_t)ctx->tloc_off[ctx->n_elem];
    hipLaunchKernelGGL(k_resid_face, dim3(ctx->n_face), dim3(128), 0, s, ctx->dm, (const double *)ruh, fpart);
    hipLaunchKernelGGL(k_resid_final, dim3(1), dim3(256), 0, s, (const double *)part, ctx->n_elem,
                       (const double *)fpart, ctx->n_face, out);
    return (int)hipGetLastError();
}

int launch_admissible(const hdg_ctx *ctx, double alpha, const double *U, const double *dQU, int *flag, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_flag, dim3(1), dim3(1), 0, s, flag);
    hipLaunchKernelGGL(k_admissible, dim3(ctx->n_elem), dim3(256), 0, s, ctx->dm, alpha, ctx->phys.gamma, U, dQU,
                       flag);
    return (int)hipGetLastError();
}

int launch_recover(const hdg_ctx *ctx, int prec, int e0, int ne, const double *E, const double *dUhat, double *dQU,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_recover, dim3(ne), dim3(kRT), 0, s, ctx->dm, e0, prec == HDG_FP64 ? 1 : 0, E,
                       (const double *)nullptr, dUhat, dQU);
    return (int)hipGetLastError();
}

int launch_recover_x(const hdg_ctx *ctx, int e0, int ne, const double *X, const double *dUhat, double *dQU,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_recover, dim3(ne), dim3(kRT), 0, s, ctx->dm, e0, 0, (const double *)nullptr, X, dUhat, dQU);
    return (int)hipGetLastError();
}

int launch_store_x(const hdg_ctx *ctx, int e0, int ne, const double *E, double *X, hipStream_t s) {
    hipLaunchKernelGGL(k_store_x, dim3((ctx->max_n + kStoreXRows - 1) / kStoreXRows, ne), dim3(256), 0, s, ctx->dm, e0,
                       E, X);
    return (int)hipGetLastError();
}

}  // namespace hdg
