// Internal declarations of libhdg: context, device tables, kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <vector>

#include "../../include/hdg.h"

namespace hdg {

constexpr int kMaxP = 4;

// ---------------------------------------------------------------- 1-D tables
// Lagrange polynomials of the Gauss-Lobatto nodes evaluated at Gauss points:
//   L(p, q, a, s) = l^p_a(x^{q+2}_s)     p, q in 1..4 (basis degree, rule of degree q)
//   D(p, a, g)    = (l^p_a)'(x^{p+2}_g)
//   W(nq, g)      = Gauss weight, nq in 3..6
constexpr int kTblL = 0;
constexpr int kTblD = kTblL + 16 * 30;
constexpr int kTblW = kTblD + 4 * 30;
constexpr int kTblSize = kTblW + 4 * 6;
__host__ __device__ inline int tbl_L(int p, int q, int a, int s) { return kTblL + ((p - 1) * 4 + (q - 1)) * 30 + a * 6 + s; }
__host__ __device__ inline int tbl_D(int p, int a, int g) { return kTblD + (p - 1) * 30 + a * 6 + g; }
__host__ __device__ inline int tbl_W(int nq, int g) { return kTblW + (nq - 3) * 6 + g; }

// Per-element quadrature-point data written by the point kernels (doubles):
//   volume  vjac [c 5][s 20][d 4][g]   coefficient of phi_k and of the reference
//                                      derivatives of phi_i in row u_c, column field s
//           vres [r 20][d 4][g]        residual coefficients of row field r
//   face lf (lf = 0..5, points of that face)
//           fjac [c 5][slot 25][s]     d(fh_c dS)/d(u 0..4, q 5..19, uh 20..24), weights included
//           fres [c 5][s]              fh_c dS
//           bres [c 5][s]              boundary residual w |N| b^_c (boundary faces)
//           fuh  [c 5][s]              uh_c
//           bjac [c 5][slot 25][s]     d(b^_c)/d(u, q, uh), weights included (boundary faces)
constexpr int kVJac = 400, kVRes = 80, kFJac = 125, kFPer = 265;

// Device view of a context, passed by value to kernels.
struct DevMesh {
    int n_elem, n_face;
    const int *elem_p;         // [n_elem]
    const int *face_p;         // [n_face]
    const int *elem_face;      // [n_elem][6]
    const int *face_bc;        // [n_face]
    const int *toff;           // [n_elem][7] element-local trace offsets per local face
    const int64_t *node_off;   // [n_elem+1]
    const int64_t *face_off;   // [n_face+1]
    const int64_t *E_off;      // [n_elem+1]
    const int64_t *SK_off;     // [n_elem+1]
    const int64_t *asm_off;    // [n_elem+1]
    const int64_t *qp_off;     // [n_elem+1]
    const int64_t *asmsys_off; // [n_elem+1] Schwarz inversion systems [S_r | I] (m x ld entries, m = asm_pad(f))
    const int64_t *tloc_off;   // [n_elem+1] prefix sums of f_e (element-local trace vectors)
    const int64_t *m32_off;    // [n_elem+1] FP32 interior systems [A | B R_qu] (n x e_ld floats)
    const int64_t *x_off;      // [n_elem+1] X = A^{-1}[B | R_qu] (n x x_ld doubles)
    const int64_t *vgeo_off;   // [n_elem+1]  volume geometry: [10][Nq] = W, G00..G22 (G = J^{-1})
    const int64_t *fgeo_off;   // [n_elem*6+1] face geometry: [4][Nqf] = w N_x, w N_y, w N_z, w |N|
    const double *vgeo;
    const double *fgeo;
    const double *tbl;         // kTblSize doubles
    // block-sparse trace operator
    const int *bsr_row_ptr;    // [n_face+1]
    const int *bsr_col;        // [nnzb]
    const int64_t *bsr_val_off;// [nnzb+1]
    const int *blk_src_ptr;    // [nnzb+1] contributions to each block
    const int *blk_src;        // [n][3]: elem, local face a (row), local face b (col)
    const int *face_src_ptr;   // [n_face+1] elements touching each face
    const int *face_src;       // [n][2]: elem, local face
    const int *asm_blk;        // [n_elem][36]: bsr block index of (face a, face b)
    // artificial-viscosity smoothing: element corners grouped into vertex
    // classes (vertices identified through every two-sided face, periodic
    // pairs included)
    int n_vclass;
    const int *av_corner;      // [n_elem][8] vertex class of each corner (tensor order)
    const int *av_src_ptr;     // [n_vclass+1]
    const int *av_src;         // elements touching each class, ascending
};

struct Phys {
    double gamma, prandtl, reynolds, mach, tau, dt, alpha;
    int visc_law;
};

// Element-system row stride (doubles): n + f + 1 rounded up to a multiple of 8.
__host__ __device__ inline int64_t e_ld(int n, int f) { return ((int64_t)(n + f + 1) + 7) / 8 * 8; }
// Size of an element's Schwarz inversion system: f rounded up to a multiple of 4
// (extra unknowns are decoupled), so that every panel width and column offset
// allows 16-byte FP32 and FP64 accesses.
__host__ __device__ inline int asm_pad(int f) { return (f + 3) & ~3; }
// Row stride of X (doubles): f + 1 rounded up to a multiple of 8.
__host__ __device__ inline int64_t x_ld(int f) { return ((int64_t)(f + 1) + 7) / 8 * 8; }

}  // namespace hdg

struct hdg_ctx {
    int device = 0;
    int n_elem = 0, n_face = 0;
    hdg::Phys phys{};
    int max_n = 0, max_f = 0, max_b = 0, max_p = 0;
    int n_vclass = 0;  // vertex classes of the artificial-viscosity smoothing
    bool uniform_p = true;
    bool repeated_face = false;  // some element meets the same face twice
    // whether every block column starts on a 128-byte line: the face blocks of
    // S (b_F doubles) and the Schwarz inverses (f_e doubles, f_e floats)
    bool face_cols_aligned = true, asm_cols_aligned64 = true, asm_cols_aligned32 = true;
    std::vector<int> elem_p, face_p, elem_face, face_elem, face_bc, toff, elem_n, elem_f;
    std::vector<int64_t> node_off, face_off, E_off, SK_off, asm_off, qp_off, vgeo_off, fgeo_off, asmsys_off,
        tloc_off, m32_off, x_off;
    std::vector<int64_t> bsr_row_ptr64, bsr_col64, bsr_val_off;
    std::vector<int> bsr_row_ptr, bsr_col;
    hdg::DevMesh dm{};
    std::vector<void *> allocations;  // device buffers owned by the context
    std::map<int, int> update_tile;   // n (0: every n) -> rows of the trailing-update tile (128 or 256)
};

namespace hdg {
// kernel launchers (return hipError_t as int)
int launch_element_system(const hdg_ctx *ctx, int e0, int ne, const double *Q, const double *U,
                          const double *Un, const double *Uhat, const double *nu, const double *Ub,
                          double *E, double *qp, hipStream_t s);
int launch_condense_fp64(const hdg_ctx *ctx, int e0, int ne, double *E, double *SK, int *info,
                         void *work, hipStream_t s);
int launch_condense_mixed(const hdg_ctx *ctx, int e0, int ne, int refine, double *E, double *SK,
                          int *info, void *work, hipStream_t s);
size_t condense_mixed_work_bytes(const hdg_ctx *ctx, int e0, int ne);
int launch_condense_fast(const hdg_ctx *ctx, int e0, int ne, double *E, double *SK, int *info, void *work,
                         hipStream_t s);
size_t condense_fast_work_bytes(const hdg_ctx *ctx, int e0, int ne);
size_t bordered_lu_work(const hdg_ctx *ctx, int ne);
int run_asm_inversion(const hdg_ctx *ctx, int prec, void *sys, int *info, void *work, hipStream_t s);
int launch_assemble(const hdg_ctx *ctx, const double *SK, double *S, double *g, hipStream_t s);
int launch_matvec(const hdg_ctx *ctx, const double *S, const double *x, double *y, hipStream_t s);
// attainable-peak probes (k_peak.hip)
int launch_peak_mfma(int fp_bits, int n_wg, int iters, double one, void *sink, hipStream_t s);
int launch_peak_read(const void *src, size_t bytes, unsigned *sink, hipStream_t s);
int launch_peak_copy(const void *src, void *dst, size_t bytes, hipStream_t s);
int launch_asm_setup(const hdg_ctx *ctx, int prec, const double *S, void *Sinv, int *info,
                     void *work, hipStream_t s);
size_t asm_setup_work_bytes(const hdg_ctx *ctx, int prec);
size_t schwarz_ws_bytes(const hdg_ctx *ctx, int prec);
int launch_asm_apply(const hdg_ctx *ctx, int prec, const void *Sinv, const double *r, double *z,
                     void *work, hipStream_t s);
size_t asm_apply_work_bytes(const hdg_ctx *ctx);
// hdg_asm_block_apply_noalloc: a per-device library array holds zloc.
constexpr size_t kAsmScratchDoubles = HDG_ASM_NOALLOC_MAX_DOUBLES;  // 32 MiB
int asm_scratch_init(int device);
int launch_asm_apply_noalloc(const hdg_ctx *ctx, int prec, const void *Sinv, const double *r, double *z,
                             hipStream_t s);
int launch_gmres(const hdg_ctx *ctx, int prec, const double *S, const void *Sinv, const double *g,
                 const double *x0, int m, double *x, double *hist, void *work, hipStream_t s);
size_t rb_work_bytes(const hdg_ctx *ctx, int nb_max);
int launch_rb_guess(const hdg_ctx *ctx, int nb, const double *W, const double *Z, const double *g, double *x0,
                    void *work, hipStream_t s);
int launch_rb_insert(const hdg_ctx *ctx, const double *S, const double *w_new, int slot, double *W, double *Z,
                     hipStream_t s);
int launch_state_update(const hdg_ctx *ctx, double alpha, const double *dQU, const double *dUhat, double *Q,
                        double *U, double *Uhat, hipStream_t s);
int launch_lincomb(int k, const double *const *v, const double *c, double *out, int64_t n, hipStream_t s);
size_t resid_work_bytes(const hdg_ctx *ctx);
int launch_resid_elem(const hdg_ctx *ctx, int e0, int ne, const double *E, void *work, hipStream_t s);
int launch_resid_norm(const hdg_ctx *ctx, void *work, double *out, hipStream_t s);
int launch_admissible(const hdg_ctx *ctx, double alpha, const double *U, const double *dQU, int *flag,
                      hipStream_t s);
size_t gmres_work_bytes(const hdg_ctx *ctx, int m);
struct AvParams {
    double c_av, h_m, eps, s_max, rho_min, p_min;
    int smooth_iters;
};
size_t av_work_bytes(const hdg_ctx *ctx);
void gll_nodes(int p, double *r);  // Gauss-Lobatto nodes of degree p on [-1, 1]
int launch_av_field(const hdg_ctx *ctx, const AvParams &ap, const double *U, const double *Q, double *nu_raw,
                    double *nu, void *work, hipStream_t s);
int launch_recover(const hdg_ctx *ctx, int prec, int e0, int ne, const double *E,
                   const double *dUhat, double *dQU, hipStream_t s);
int launch_store_x(const hdg_ctx *ctx, int e0, int ne, const double *E, double *X, hipStream_t s);
int launch_recover_x(const hdg_ctx *ctx, int e0, int ne, const double *X, const double *dUhat, double *dQU,
                     hipStream_t s);
}  // namespace hdg
