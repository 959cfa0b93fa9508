/*
 * hdg.h -- C ABI of libhdg: the element-local hot path of an HDG
 * Newton-GMRES solver for the compressible Navier-Stokes equations on one
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Welter, Collin, Nguyen, Peraire, "A Massively Parallel Hybridizable
 * Discontinuous Galerkin Solver for Direct Numerical Simulation of
 * Compressible Flows on GPUs".  Section references below are to that paper.
 *
 * One Newton iteration of a DIRK stage (sections 2.4-3.3) is
 *   hdg_local_residual_jacobian   element residuals and Jacobian blocks
 *   hdg_condense                  static condensation per element
 *   hdg_assemble_trace            assembly of the condensed trace system
 *   hdg_asm_setup                 additive-Schwarz local inverses
 *   hdg_gmres                     left-preconditioned GMRES on S dUhat = g
 *      (uses hdg_face_matvec and hdg_asm_block_apply)
 *   hdg_recover_interior          interior correction from the trace one
 *
 * Conventions shared by every call
 * --------------------------------
 * - Pointers named "host" are host memory; every other array pointer is
 *   device memory owned by the caller (the library never frees it).  The
 *   context owns only its own tables (freed by hdg_destroy).
 * - `stream` is a hipStream_t passed as void*; every call only enqueues work
 *   on it (no host synchronisation, no allocation), so calls can be captured
 *   in a HIP graph.  NULL is the default stream.
 * - Return value: HDG_OK, or a negative hdg_status.  Arguments are checked
 *   on the host before anything is enqueued; a failed launch returns
 *   HDG_ERR_DEVICE.  Numerical failures never synchronise: they are written
 *   to device `info` arrays.
 * - Unknowns (nondimensional, rho_0 = |v_0| = L = T_0 = 1):
 *     U  : conserved variables u = (rho, rho v1, rho v2, rho v3, rho E)
 *     Q  : gradient q = grad u, q_{c,j} = d u_c / d x_j   (eq. mixed-variable)
 *     Uh : single-valued face trace of u                   (eq. spaces)
 * - Element e has degree p_e (1..4), N_p = (p_e+1)^3 Gauss-Lobatto nodes in
 *   tensor order (x fastest).  Face F has degree p_F = max of its sides and
 *   N_fp = (p_F+1)^2 trace nodes.  Volume quadrature: (p_e+2)^3 Gauss
 *   points; face quadrature: (p_F+2)^2 Gauss points.
 * - Packed node arrays (layout [e][field][node], elements back to back;
 *   element e starts at field_count * node_off[e]):
 *     Q [15 N_p] fields 3c+j;  U, Un [5 N_p];  nu [N_p];  dQU [20 N_p]
 *     (dQU fields 0..14 are dq_{c,j}, 15..19 are du_c).
 * - Packed face arrays ([F][c][node], face F starts at face_off[F]):
 *     Uhat, Ub, g, dUhat, x, y, r, z.  Total length N_uh = face_off[n_face].
 * - Element-local trace order: local faces -x,+x,-y,+y,-z,+z, each
 *   [c][node]; f_e = sum over the 6 faces of 5 N_fp; n_e = 20 N_p.
 * - Element system E^K (one per element, ROW-major, n+f rows of stride
 *   ldE = n+f+1 rounded up to a multiple of 8; columns n+f+1 .. ldE-1 are
 *   padding, written as 0), the linearised local problem of
 *   eq. newton-local-block bordered by the element's trace equations:
 *         [ A  B  R_qu ]   rows 0..n-1     A = d(R_q,R_u)/d(Q,U)   (n x n)
 *         [ C  D  R_uh ]   rows n..n+f-1   B = d(R_q,R_u)/d(Uh^K)  (n x f)
 *                                          C = d(R_uh^K)/d(Q,U)    (f x n)
 *                                          D = d(R_uh^K)/d(Uh^K)   (f x f)
 *   Element e's system starts at E_off[e] doubles (relative to E_off[e0]
 *   for a chunk starting at element e0).
 * - Condensed element output SK (per element, column-major f x (f+1)):
 *   [ S^K | g^K ] with S^K = D - C A^{-1} B and g^K = -R_uh + C A^{-1} R_qu
 *   (eqs. local-elimination, schur-trace).  Element e at SK_off[e].
 * - Assembled trace operator S: block-sparse rows, one block row per face,
 *   block (F, F') of size (5 N_fp(F)) x (5 N_fp(F')) stored column-major at
 *   bsr_val_off[k] for k in bsr_row_ptr[F] .. bsr_row_ptr[F+1]-1, column
 *   face bsr_col[k] (ascending).  Pattern built by hdg_create.  Every
 *   bsr_val_off[k] is a multiple of 16 (blocks start on 128-byte lines); the
 *   entries between a block's end and the next offset are zero after
 *   hdg_assemble_trace.
 * - Layout arrays are obtained with hdg_layout().
 */
#ifndef HDG_H
#define HDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hdg_ctx hdg_ctx;

typedef enum {
    HDG_OK = 0,
    HDG_ERR_INVALID_ARGUMENT = -1,
    HDG_ERR_UNSUPPORTED = -2,
    HDG_ERR_OUT_OF_MEMORY = -3,
    HDG_ERR_DEVICE = -4,
    HDG_ERR_WORKSPACE = -5
} hdg_status;

/* Arithmetic of the element condensation and of the Schwarz blocks. */
typedef enum {
    HDG_FP64 = 0,   /* FP64 throughout                                          */
    HDG_MIXED = 1,  /* FP32 LU / triangular solves with FP32 accumulation,
                       FP64-residual iterative refinement of A^{-1}[B|R_qu],
                       FP64 Schur product; Schwarz inverses stored in FP32     */
    HDG_MIXED_FAST = 2 /* hdg_condense only (and the recovery after it): the whole
                       bordered system factored in FP32, the Schur complement
                       formed by the FP32 trailing updates with FP32
                       accumulation, no refinement.  Error about cond(A) u_32:
                       reported beside HDG_MIXED, not accurate to 1e-10        */
} hdg_precision;

/* Mesh: conforming hexahedra, all elements identically oriented (every face is
 * seen with the same tangential axes from both sides).  Host memory, copied. */
typedef struct hdg_mesh_desc {
    int n_elem, n_face, n_vert;
    const double *vert_xyz;      /* host [n_vert][3]                                   */
    const int *elem_vert;        /* host [n_elem][8], tensor order (x fastest)        */
    const int *elem_face;        /* host [n_elem][6], faces -x,+x,-y,+y,-z,+z          */
    const int *face_elem;        /* host [n_face][2][2]: (elem, local face) of side 0
                                    and side 1; side 1 = (-1,-1) on a boundary face.
                                    The face normal points out of side 0.              */
    const signed char *face_bc;  /* host [n_face]: boundary type, see below             */
    const signed char *elem_p;   /* host [n_elem]: degree 1..4                         */
    const double *elem_geom;     /* host [n_elem][27][3] or NULL: curved (triquadratic)
                                    geometry, the element's map through 27 nodes in
                                    tensor order (x fastest) at reference coordinates
                                    -1, 0, 1; NULL = the trilinear map of the vertices.
                                    Vertices still define the topology; nodes on shared
                                    faces must coincide (section 2.2: curved elements). */
} hdg_mesh_desc;

/* Boundary types (face_bc of a one-sided face; the weak boundary statement
 * b^ of eq. hdg-trace replaces the numerical flux in the face's trace
 * equations, integrated against mu with the face's |N| dS; the conservation
 * equations keep the numerical flux fh of eq. num-flux-hdg evaluated with the
 * trace), following the boundary-condition paragraph of section 2.1:
 *   HDG_BC_STATE      b^ = uh - ub          prescribed exterior state (far field,
 *                                           supersonic inflow); reads Ub
 *   HDG_BC_EXTRAP     b^ = uh - u           interior state extrapolated
 *                                           (supersonic outflow)
 *   HDG_BC_WALL_T     b^ = (rho^ - rho, m^, rho^E^ - rho^ e_w)
 *                                           no-slip isothermal wall; e_w = the internal
 *                                           energy of ub (reads Ub)
 *   HDG_BC_WALL_ADIAB b^ = (rho^ - rho, m^, fh_energy)
 *                                           no-slip adiabatic wall (no energy flux)
 *   HDG_BC_SYMMETRY   b^ = (rho^ - rho, m^ - (I - n n^T) m, rho^E^ - rhoE)
 *                                           zero normal velocity, tangential state
 *                                           from the interior                        */
enum { HDG_BC_NONE = 0, HDG_BC_STATE = 1, HDG_BC_EXTRAP = 2, HDG_BC_WALL_T = 3, HDG_BC_WALL_ADIAB = 4,
       HDG_BC_SYMMETRY = 5 };

/* Physical and time-discretisation constants (section 2, section 5). */
typedef struct hdg_phys {
    double gamma;     /* ratio of specific heats                                   */
    double prandtl;   /* Pr, heat flux gamma mu / (Re Pr) de/dx (eq. thermal-conductivity) */
    double reynolds;  /* viscosity mu(T) / Re                                      */
    double mach;      /* T = gamma (gamma-1) M^2 e                                 */
    double tau;       /* HDG stabilisation tau_h = tau * I (eq. num-flux-hdg)       */
    double dt;        /* time step multiplying N in eq. fully-discrete-local        */
    double alpha;     /* DIRK diagonal d_ii multiplying M (U - U^n)                */
    int visc_law;     /* 0: mu = 1; 1: mu = 1.4042 T^1.5 / (T + 0.40417) (eq. tgv-sutherland) */
} hdg_phys;

/* Create a context on the current HIP device: copies the mesh, computes the
 * quadrature tables and geometry (inverse Jacobians, weights, area-weighted
 * normals), the assembly maps and the block-sparse pattern.  Blocking; the
 * only call that allocates device memory.  Returns HDG_ERR_INVALID_ARGUMENT
 * for an inconsistent mesh (bad indices, degree outside 1..4, a face whose two
 * sides are not opposite local faces, or a non-positive Jacobian). */
int hdg_create(const hdg_mesh_desc *mesh, const hdg_phys *phys, hdg_ctx **out);
void hdg_destroy(hdg_ctx *ctx);
const char *hdg_status_string(int status);

/* Layout queries: hdg_layout copies a host array of int64 into dst (host). */
typedef enum {
    HDG_LAYOUT_NODE_OFF = 0,    /* [n_elem+1] node offsets                            */
    HDG_LAYOUT_FACE_OFF = 1,    /* [n_face+1] face trace offsets (doubles)            */
    HDG_LAYOUT_E_OFF = 2,       /* [n_elem+1] element-system offsets (doubles)        */
    HDG_LAYOUT_SK_OFF = 3,      /* [n_elem+1] condensed-output offsets (doubles)      */
    HDG_LAYOUT_BSR_ROW_PTR = 4, /* [n_face+1]                                         */
    HDG_LAYOUT_BSR_COL = 5,     /* [nnzb]                                             */
    HDG_LAYOUT_BSR_VAL_OFF = 6, /* [nnzb+1] block offsets (doubles)                   */
    HDG_LAYOUT_ASM_OFF = 7,     /* [n_elem+1] Schwarz block offsets (entries, multiples
                                   of 32: blocks start on 128-byte lines; the entries
                                   between blocks are zero after hdg_asm_setup)        */
    HDG_LAYOUT_ELEM_N = 8,      /* [n_elem] n_e                                       */
    HDG_LAYOUT_ELEM_F = 9,      /* [n_elem] f_e                                       */
    HDG_LAYOUT_X_OFF = 10       /* [n_elem+1] retained-X offsets (doubles): element e's
                                   X is row-major n_e x x_ld_e, x_ld_e = f_e + 1 rounded
                                   up to a multiple of 8                               */
} hdg_layout_kind;
int hdg_layout(const hdg_ctx *ctx, int kind, int64_t *dst, int64_t capacity);
/* Length of a layout array (so the caller can size dst). */
int64_t hdg_layout_length(const hdg_ctx *ctx, int kind);

/* Block-sparse pattern of the assembled trace operator S of eq. schur-trace
 * (section 3.2): face F's row holds one block per face G that shares an element
 * with F.  *nnzb receives the number of blocks; *row_ptr_dev a device array of
 * int32 [n_face+1], *col_dev a device array of int32 [nnzb] (ascending G within
 * a row): the same values as HDG_LAYOUT_BSR_ROW_PTR and HDG_LAYOUT_BSR_COL.  The
 * arrays belong to the context, are read-only and stay valid until hdg_destroy.
 * Any output pointer may be NULL.  No device work; HDG_ERR_INVALID_ARGUMENT
 * for a null context. */
int hdg_bsr_pattern(const hdg_ctx *ctx, int *nnzb, const int **row_ptr_dev, const int **col_dev);

/* Attainable peaks, for roofline fractions against what this chip reaches
 * beside its datasheet figures (measurement helpers, not steps of the method).
 * hdg_peak_mfma: n_wg (1 .. 1048576) workgroups of 256 threads; each of their
 * waves issues iters (>= 1) x 8 independent 16x16x4 matrix-core products from
 * register operands equal to `one`, FP64 for fp_bits = 64, FP32 for 32:
 * n_wg * 4 * iters * 8 * 2048 flop per call.  sink: device, n_wg * 256 values
 * of that type, caller-owned; each receives 128 * iters * one^2 (exact for
 * one = 1 while 4 * iters < 2^24 in FP32).  hdg_peak_read: reads `bytes` (a
 * positive multiple of 16) from src (device, 16-byte aligned) and XORs every
 * 32-bit word into *sink (device, one uint32 the caller zeroes first).
 * hdg_peak_copy: copies `bytes` (a positive multiple of 16) from src to dst
 * (device, 16-byte aligned, not overlapping): 2 * bytes of memory traffic.
 * All are asynchronous on `stream`; HDG_ERR_INVALID_ARGUMENT for other
 * arguments. */
int hdg_peak_mfma(int fp_bits, int n_wg, int iters, double one, void *sink, void *stream);
int hdg_peak_read(const void *src, size_t bytes, unsigned *sink, void *stream);
int hdg_peak_copy(const void *src, void *dst, size_t bytes, void *stream);

/* Workspace sizes in bytes (caller allocates, 256-byte aligned).  `op` is the
 * entry point: 0 hdg_local_residual_jacobian and 1 hdg_condense (for a chunk
 * of ne elements starting at e0), 2 hdg_asm_setup, 3 hdg_asm_block_apply,
 * 4 hdg_gmres / hdg_gmres_x0 (with Krylov dimension m = ne), 5 hdg_rb_guess
 * (with ne = the largest basis size used), 6 hdg_residual_gather /
 * hdg_residual_norm, 7 hdg_av_field. */
int hdg_workspace_size(const hdg_ctx *ctx, int op, int prec, int e0, int ne, size_t *bytes);

/*
 * Element residuals and Jacobians (steps of eqs. hdg-grad, hdg-cons with the
 * DIRK mass term of eq. fully-discrete-local, hdg-trace; the flux of
 * eq. num-flux-hdg with tau_h = tau I; fluxes of eqs. convective-flux,
 * viscous-flux, stress-heat, av-total; Jacobians of eq. newton-linearization).
 * For elements e0 .. e0+ne-1 writes E^K completely (every entry), where
 *   R_q[(c,j),i] = int_K q_cj phi_i + int_K u_c d_j phi_i - int_dK uh_c phi_i n_j
 *   R_u[c,i]     = alpha int_K (u-u^n)_c phi_i - dt int_K (F^c - F^v)_cj d_j phi_i
 *                  + dt int_dK fh_c phi_i
 *   R_uh^K[F,c,a]= int_F fh_c mu_a            (interior / periodic faces)
 *                = int_F b^_c mu_a            (boundary faces, b^ per face_bc above)
 *   fh = (F^c(uh) - F^v(uh, q)) . n + tau (u - uh),  F^v includes nu q.
 * nu is frozen (no derivative).  Ub is read only on faces of types
 * HDG_BC_STATE and HDG_BC_WALL_T (may be NULL when the mesh has none).  E points at element e0's system.  `work`
 * (hdg_workspace_size op 0) holds the quadrature-point fluxes and Jacobians
 * (the point kernel's output, read by the assembly kernel).
 */
int hdg_local_residual_jacobian(hdg_ctx *ctx, int e0, int ne,
                                const double *Q, const double *U, const double *Un,
                                const double *Uhat, const double *nu, const double *Ub,
                                double *E, void *work, size_t work_bytes, void *stream);

/*
 * Tile shape of the trailing update of the blocked LU (the dominant kernel of
 * hdg_condense and of the Schwarz inversion), per size of system: systems with
 * n pivot columns (n = 20 N_p for element systems; n = 0 sets the default for
 * every size) use tiles of tile_rows x 128 (tile_rows 128 or 256; default
 * 128).  Chosen by measurement (the Python pipeline's autotuner times both on
 * the device).  A chunk mixing sizes uses the setting of its largest n.
 * hdg_get_update_tile returns the rows in effect for n.
 */
int hdg_set_update_tile(hdg_ctx *ctx, int n, int tile_rows);
int hdg_get_update_tile(const hdg_ctx *ctx, int n);

/*
 * Static condensation (eqs. local-elimination, schur-trace) of elements
 * e0 .. e0+ne-1.  E (element e0's system first) is overwritten:
 *  HDG_FP64: partial LU with partial pivoting of the first n columns of E
 *    (pivots chosen among rows 0..n-1), the elimination carried through the
 *    trace rows and the [B | R_qu] columns.  Afterwards rows 0..n-1 hold U (upper
 *    triangle of the n x n block) and L^{-1} P [B | R_qu]; rows n.. hold
 *    [S^K | -g^K].
 *  HDG_MIXED_FAST: as HDG_FP64 but in FP32 (an FP32 copy of the systems in the
 *    workspace); S^K and g^K carry the FP32 rounding; rows 0..n-1 of E are then
 *    overwritten with the FP32 factors converted to FP64 (for the recovery).
 *  HDG_MIXED: A is factorised in FP32 in the workspace, X = A^{-1}[B | R_qu] is
 *    refined `refine_steps` (>= 1) times with FP64 residuals [B|R_qu] - A X, S^K
 *    and g^K are formed with FP64 products; X is then stored in place of
 *    [B | R_qu] (rows 0..n-1, columns n..n+f).
 * SK (all elements, element e at SK_off[e]) receives [S^K | g^K].
 * info[e] (device, all elements) = 0, or k+1 if the k-th pivot was zero or
 * not finite (the element's outputs are then undefined; the other elements'
 * outputs are unaffected).  A NaN that is never a pivot candidate's maximum is
 * not reported: it propagates to that element's outputs.
 */
int hdg_condense(hdg_ctx *ctx, int prec, int refine_steps, int e0, int ne, double *E,
                 double *SK, int *info, void *work, size_t work_bytes, void *stream);

/*
 * Assembly of S = sum_K P_K^T S^K P_K and g = sum_K P_K^T g^K (eq. schur-trace)
 * into the block-sparse S (all blocks written) and g.  Each block and face is
 * a gather over its element contributions in a fixed order (bit-reproducible,
 * no atomics).  Needs SK of every element.
 */
int hdg_assemble_trace(hdg_ctx *ctx, const double *SK, double *S_bsr, double *g, void *stream);

/*
 * y = S x with the assembled condensed trace operator S of eq. schur-trace
 * (section 3.2: the operator is assembled once per Newton iteration and
 * applied in every Krylov iteration).  S_bsr in the block-sparse layout above
 * (all blocks of the pattern); x, y face arrays of length N_uh; x and y must
 * not alias.  Reads S once: bound by HBM bandwidth.
 */
int hdg_face_matvec(hdg_ctx *ctx, const double *S_bsr, const double *x, double *y, void *stream);

/*
 * One-level additive Schwarz set-up (eq. additive-schwarz): for every element
 * r, S_r = R_r S R_r^T (its six faces' blocks of the assembled S) is inverted
 * by LU with partial pivoting; the inverse is stored in Sinv at ASM_off[r]
 * entries, column-major f_r x f_r, as double (HDG_FP64) or float (HDG_MIXED).
 * info[r] = 0 or k+1 on a zero pivot.
 */
int hdg_asm_setup(hdg_ctx *ctx, int prec, const double *S_bsr, void *Sinv, int *info,
                  void *work, size_t work_bytes, void *stream);

/*
 * z = sum_r R_r^T S_r^{-1} R_r r (eq. additive-schwarz): restriction to each
 * element's faces, the local solve with the stored inverse (FP64 data, or FP32
 * data with FP64 accumulation), and prolongation summed over the elements
 * sharing a face in a fixed order.
 */
int hdg_asm_block_apply(hdg_ctx *ctx, int prec, const void *Sinv, const double *r, double *z,
                        void *work, size_t work_bytes, void *stream);

/*
 * hdg_asm_block_apply for callers that cannot allocate device memory (code
 * under HIP stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same z = sum_r R_r^T S_r^{-1} R_r r with the same kernels, but
 * the element-local corrections live in a library-owned device array of
 * HDG_ASM_NOALLOC_MAX_DOUBLES doubles (32 MiB) instead of a caller workspace.
 * Each GPU the library runs on holds one such array from hdg_create until the
 * process ends.  Returns HDG_ERR_WORKSPACE when the mesh needs more than that
 * (sum over elements of f_e > HDG_ASM_NOALLOC_MAX_DOUBLES, e.g. more than
 * 5592 elements of degree 4).  Allocates nothing.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams,
 * other threads, other contexts) race and must be serialised by the caller.
 */
#define HDG_ASM_NOALLOC_MAX_DOUBLES 4194304
int hdg_asm_block_apply_noalloc(hdg_ctx *ctx, int prec, const void *Sinv, const double *r, double *z,
                                void *stream);

/*
 * One cycle of left-preconditioned GMRES(m) on S dUhat = g, x0 = 0
 * (section 3.2): Arnoldi with classical Gram-Schmidt applied twice, Givens
 * rotations and the triangular solve on the device, all FP64.  res_hist
 * (device, m+1 doubles) receives ||M^{-1}(g - S x_j)||_2, j = 0..m.
 * m in 1..200.
 */
int hdg_gmres(hdg_ctx *ctx, int prec, const double *S_bsr, const void *Sinv, const double *g,
              int m, double *dUhat, double *res_hist, void *work, size_t work_bytes,
              void *stream);

/*
 * GMRES(m) started from an initial guess x0 (device, N_uh): as hdg_gmres, but
 * the cycle minimises ||M^{-1}(g - S x)||_2 over x0 + K_m(M^{-1} S, r0) with
 * r0 = M^{-1}(g - S x0) (section 3.2; the reduced basis of section 3.4 supplies
 * x0).  res_hist[0] = ||r0||.  dUhat may alias x0.  Workspace op 4.
 */
int hdg_gmres_x0(hdg_ctx *ctx, int prec, const double *S_bsr, const void *Sinv, const double *g, const double *x0,
                 int m, double *dUhat, double *res_hist, void *work, size_t work_bytes, void *stream);

/*
 * Reduced-basis initial guess (section 3.4, eq. rb-min).  W and Z are device
 * arrays of column vectors of length N_uh (column j at j * N_uh): W holds
 * previously accepted trace corrections w_j and Z their products z_j = S w_j,
 * taken with the trace operator of the iteration that accepted them.  With the
 * first nb columns:
 *   c = argmin_c || g - Z c ||_2,   x0 = W c.
 * Computed by classical Gram-Schmidt QR of Z (two projections per column) and
 * c = R^{-1} Q^T g; a column whose part orthogonal to the previous ones is
 * below 1e-12 of its norm is dependent on them and gets c_j = 0 (the kept
 * columns span the same space, so the minimal residual is the same).  nb = 0
 * gives x0 = 0 (W, Z, work may be NULL).  0 <= nb <= HDG_RB_MAX.  Workspace
 * op 5 with ne = nb (or the largest nb used).
 */
#define HDG_RB_MAX 32
int hdg_rb_guess(hdg_ctx *ctx, int nb, const double *W, const double *Z, const double *g, double *x0, void *work,
                 size_t work_bytes, void *stream);

/*
 * Insert an accepted trace correction into the reduced basis (section 3.4):
 * the window of at most nb_max columns is first-in first-out.  W[:, *head] =
 * w_new and Z[:, *head] = S w_new (one application of the trace operator),
 * then *head = (*head + 1) mod nb_max and *count = min(*count + 1, nb_max),
 * so that once the window is full the oldest column is the one replaced.
 * count and head are host ints (in/out); 1 <= nb_max <= HDG_RB_MAX.
 */
int hdg_rb_insert(hdg_ctx *ctx, const double *S_bsr, const double *w_new, int nb_max, int *count, int *head,
                  double *W, double *Z, void *stream);

/*
 * Newton update of the stage state (eq. newton-update): Q += alpha dQ,
 * U += alpha dU (dQU packed as in hdg_recover_interior) and Uhat += alpha dUhat.
 */
int hdg_state_update(hdg_ctx *ctx, double alpha, const double *dQU, const double *dUhat, double *Q, double *U,
                     double *Uhat, void *stream);

/*
 * Admissibility of the damped update (0 < alpha <= 1 in eq. newton-update):
 * flag (device int) = 1 if U + alpha dU has a node with non-positive density
 * or pressure, or a non-finite value; else 0.
 */
int hdg_state_admissible(hdg_ctx *ctx, double alpha, const double *U, const double *dQU, int *flag, void *stream);

/*
 * out = sum_{i<k} coef[i] v[i] over n doubles (1 <= k <= 8; v is a host array
 * of device pointers, coef host): the stage combinations of the DIRK method,
 * eqs. dirk-stage (the lagged mass term) and dirk-update.  out may alias any v.
 */
int hdg_lincomb(hdg_ctx *ctx, int k, const double *const *v, const double *coef, double *out, int64_t n,
                void *stream);

/*
 * Artificial-viscosity field (eq. av-coeffs and the smoothing operator S_h of
 * section 2.1; lagged: computed from a state and then held fixed as the nu
 * input of hdg_local_residual_jacobian).  At every node of element e (degree
 * k = p_e), from U and its gradient Q:
 *   dv_i/dx_j = (q_{1+i,j} - v_i q_{0,j}) / rho,  div = dv_k/dx_k,
 *   omega = |curl v|,  c* = sqrt(gamma p* / rho*), rho* = max(rho, rho_min),
 *   p* = max(p, p_min),  Ld = max(-div, 0) (compression),  Lw = max(omega, 0),
 *   s = sqrt(h_m / k) (Ld / c*) Ld^2 / (Ld^2 + Lw^2 + eps),
 *   value = c_av min(max(s, 0), s_max);
 * nu_raw[e] = the maximum over the element's nodes (the raw elemental
 * viscosity).  Smoothing, smooth_iters >= 1 times: each vertex takes the mean
 * of the elemental values of the elements sharing it (vertices are identified
 * through every two-sided face, periodic pairs included), and between passes
 * each element takes the mean of its 8 vertex values; nu (node array) is the
 * trilinear interpolant of the final vertex values at each element's nodes, so
 * it is continuous across faces.  smooth_iters = 0 gives nu = nu_raw[e] at
 * every node of e.  nu_raw (device, n_elem) may be NULL.  Workspace op 7.
 * Readings of the paper's unspecified limiter L, c* and the smoothing are
 * these; the paper's supersonic Taylor-Green case uses c_av = 2e-3,
 * h_m = 2 pi / N and two smoothing iterations.
 */
typedef struct hdg_av_params {
    double c_av;      /* AV coefficient                                 */
    double h_m;       /* sensor length scale                            */
    double eps;       /* regularisation of the Ducros factor (> 0)     */
    double s_max;     /* upper bound of the limited sensor (> 0, may be HUGE_VAL) */
    double rho_min;   /* lower bounds of the regularised state (> 0)    */
    double p_min;
    int smooth_iters; /* 0..64                                          */
} hdg_av_params;
int hdg_av_field(hdg_ctx *ctx, const hdg_av_params *params, const double *U, const double *Q, double *nu_raw,
                 double *nu, void *work, size_t work_bytes, void *stream);

/*
 * Nonlinear residual norm of eq. nonlinear-residual.  hdg_residual_gather, for
 * elements e0 .. e0+ne-1, reads the residual columns of E just written by
 * hdg_local_residual_jacobian (before hdg_condense overwrites them) into
 * `work` (op 6); once every element is gathered, hdg_residual_norm writes
 * norms[0..2] (device) = ||R_q||_2, ||R_u||_2 and ||R_uh||_2 of the assembled
 * trace residual R_uh = sum_K P_K^T R_uh^K (eq. trace-residual), with
 * fixed-order sums (deterministic).
 */
int hdg_residual_gather(hdg_ctx *ctx, int e0, int ne, const double *E, void *work, size_t work_bytes, void *stream);
int hdg_residual_norm(hdg_ctx *ctx, void *work, size_t work_bytes, double *norms, void *stream);

/*
 * Interior recovery (eq. local-elimination): for elements e0 .. e0+ne-1,
 * d(Q,U)^K = -A^{-1} (R_qu + B dUh^K), from E as left by hdg_condense with the
 * same `prec` (HDG_FP64 and HDG_MIXED_FAST: back substitution with U;
 * HDG_MIXED: -(x_r + X_B dUh)).
 * dQU is the packed node array (all elements).
 */
int hdg_recover_interior(hdg_ctx *ctx, int prec, int e0, int ne, const double *E,
                         const double *dUhat, double *dQU, void *stream);

/*
 * Streamed condensation (the element systems of one chunk at a time; eq.
 * local-elimination).  After hdg_condense(HDG_MIXED) of elements e0 .. e0+ne-1,
 * X = A^{-1}[B | R_qu] is all that the recovery needs of their systems:
 * hdg_store_x copies it (rows 0..n-1, columns n..n+f of each system in the
 * chunk's E, laid out as for hdg_condense) into X (device, all elements,
 * element e at x_off[e] of HDG_LAYOUT_X_OFF, padding columns zeroed), after
 * which the chunk's E may be reused for the next chunk.
 * hdg_recover_interior_x is hdg_recover_interior(HDG_MIXED) reading X from that
 * store: d(Q,U)^K = -(x_r + X_B dUh^K) for elements e0 .. e0+ne-1.
 * Both only enqueue; argument errors return HDG_ERR_INVALID_ARGUMENT before any
 * launch.  E and X must not overlap.
 */
int hdg_store_x(hdg_ctx *ctx, int e0, int ne, const double *E, double *X, void *stream);
int hdg_recover_interior_x(hdg_ctx *ctx, int e0, int ne, const double *X, const double *dUhat, double *dQU,
                           void *stream);

/*
 * The whole hot path of one Newton iteration (figure "Computational workflow":
 * element residuals and Jacobians, static condensation, assembly of S and g,
 * additive-Schwarz set-up, preconditioned GMRES, interior recovery; sections
 * 2.4-3.3) as one call, and as a HIP graph.
 *
 * hdg_newton_args names every buffer of the step; all pointers except
 * chunk_e0 / chunk_ne (host) are device memory owned by the caller.  For each
 * chunk k (elements chunk_e0[k] .. chunk_e0[k]+chunk_ne[k]-1, every element in
 * exactly one chunk) the step runs hdg_local_residual_jacobian and
 * hdg_condense; then hdg_assemble_trace, hdg_asm_setup and hdg_gmres once; then
 * hdg_recover_interior per chunk.  E holds the systems of all elements
 * (element e at E_off[e]); qp_work and cond_work must be at least the
 * workspace of the largest chunk (hdg_workspace_size ops 0 and 1), asm_work
 * op 2 with asm_prec, gmres_work op 4 with ne = gmres_m.  Ub may be NULL only
 * on a mesh without faces that read Ub.  Sinv holds doubles for asm_prec =
 * HDG_FP64 and floats for HDG_MIXED.  The chunk arrays are copied.
 */
typedef struct hdg_newton_args {
    int prec;            /* condensation arithmetic, HDG_FP64 or HDG_MIXED          */
    int refine_steps;    /* HDG_MIXED: refinement steps, 1..8 (ignored for FP64)   */
    int asm_prec;        /* Schwarz inverses: HDG_FP64 (double) or HDG_MIXED (float)*/
    int gmres_m;         /* Krylov dimension, 1..200                                */
    int n_chunks;
    const int *chunk_e0; /* host [n_chunks]                                         */
    const int *chunk_ne; /* host [n_chunks]                                         */
    const double *Q, *U, *Un, *Uhat, *nu, *Ub;
    double *E;
    void *qp_work;   size_t qp_work_bytes;
    void *cond_work; size_t cond_work_bytes;
    double *SK; int *info;
    double *S_bsr, *g;
    void *Sinv; int *asm_info;
    void *asm_work;   size_t asm_work_bytes;
    void *gmres_work; size_t gmres_work_bytes;
    double *dUhat, *res_hist, *dQU;
} hdg_newton_args;

/* Enqueue the whole step on `stream` (validated first; nothing is enqueued on
 * an argument error). */
int hdg_newton_step(hdg_ctx *ctx, const hdg_newton_args *args, void *stream);

typedef struct hdg_graph hdg_graph;

/*
 * Capture the whole step in a HIP graph and instantiate it.  The step is first
 * run once on `stream` (this loads every kernel's code object, so that the
 * capture records launches only; the buffers then hold that step's results),
 * then recorded with hipStreamBeginCapture / hipStreamEndCapture on `stream`,
 * which must be a created stream (not NULL, the legacy default stream).
 * Blocking.  The graph keeps the device pointers of `args`: the buffers must
 * outlive it, and each launch recomputes the step from their current contents.
 * On success *out owns the graph (release it with hdg_graph_destroy).
 */
int hdg_graph_capture_newton(hdg_ctx *ctx, const hdg_newton_args *args, hdg_graph **out, void *stream);
/* Enqueue one replay of the captured step on `stream` (any stream, NULL too). */
int hdg_graph_launch(hdg_graph *graph, void *stream);
void hdg_graph_destroy(hdg_graph *graph);

#ifdef __cplusplus
}
#endif

#endif /* HDG_H */
