/*
 * mfbcsr -- matrix-free finite element Hamiltonian on BCSR sparse multivectors
 * for AMD Instinct MI355X (gfx950).
 *
 * What the library computes (Davydov & Kronbichler, arXiv 1907.01005):
 *
 *   Y = mask_P(X)( H X ),   S = X^T Y,   t = tr(S)
 *
 * H is the finite element Hamiltonian -1/2 Laplacian + V(x) on a box of
 * Q_p hexahedra (eq. fe_matrices), applied cell by cell with sum
 * factorisation (eq. fe_matrices_cell_based, Sec. 3.2), restricted to the
 * nodes off the homogeneous Dirichlet faces.  X is a sparse multivector in
 * BCSR layout (Sec. 3.3-3.4): row blocks are the nodes first met in each
 * 2x2x2 batch of cells along a Hilbert curve (Alg. 1), column blocks are
 * groups of orbitals sorted along the same curve (Alg. 2).  Y has the
 * pattern of X; entries of H X outside the stored blocks are dropped, as
 * the write accessor of Alg. 6 only reaches stored blocks.  S is the
 * projected matrix of eq. inner2 computed block by block as in Alg. 8, and t
 * its trace (the column-wise inner product of eq. G_ops4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every function returns an mfb_status (0 on success, negative on error)
 *    and never throws.  The message of the last error on the calling thread
 *    is returned by mfb_last_error().
 *  - Handles (mfb_mesh, mfb_mv) belong to the library; free them with the
 *    matching destroy call.  A multivector layout keeps a pointer to its
 *    mesh: the mesh must outlive it.
 *  - Device memory (values, metadata, workspace, S, trace) belongs to the
 *    caller.  The library never allocates or frees device memory; the caller
 *    keeps buffers alive while work that uses them is in flight.
 *  - Creation and host queries are synchronous and host-only (no GPU
 *    needed).  *_bind copies host-built metadata to a caller buffer with
 *    hipMemcpyAsync on the given stream.  mfb_apply_H, mfb_apply_H_tuned and
 *    mfb_tmmult only enqueue kernels on the caller's hipStream_t (passed as
 *    void*; NULL means the default stream) and return immediately.
 *  - All values are IEEE float64 in device memory.  The precision argument
 *    of mfb_apply_H only selects the arithmetic of the sum-factorisation
 *    contractions; loads, stores, quadrature scaling and accumulation into
 *    Y stay float64.
 *  - Device buffers must be 256-byte aligned (any torch CUDA allocation is).
 *  - Destinations that the apply calls accumulate into (d_Y of mfb_apply_H,
 *    mfb_apply_H_tuned and mfb_apply_op) must be coarse-grained device
 *    memory (hipMalloc, or any torch CUDA tensor).  The float64 additions
 *    into Y are hardware atomics that are not coherent on fine-grained or
 *    host-mapped memory, so such a destination gives wrong sums.
 *  - Arguments are checked before anything is enqueued: a call that returns
 *    an error has not touched any device buffer.
 *
 * Value layout of a multivector
 * -----------------------------
 * The stored blocks (r, C) are numbered in CSR order (row block r ascending,
 * column block C ascending within a row) and laid out back to back in one
 * float64 array.  Block k starts at block_offset[k] and is a dense row-major
 * rows_r x |C| matrix (row stride |C|, no padding).  Row i of block (r, C)
 * is the row row_block_start[r] + i of the multivector, whose global node is
 * dof_perm[row]; column j is column col_block_start[C] + j, whose original
 * orbital id is col_perm[column].  S is written M x M row-major in this
 * column order (S[a*M + b] pairs columns a and b).
 */
#ifndef MFBCSR_H
#define MFBCSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mfb_mesh mfb_mesh;
typedef struct mfb_mv mfb_mv;

typedef enum {
  MFB_OK = 0,
  MFB_EINVAL = -1,        /* bad argument (null pointer, size, range)          */
  MFB_EUNSUPPORTED = -2,  /* valid request the library does not implement     */
  MFB_EPATTERN = -3,      /* layout/mesh mismatch, entry outside the pattern   */
  MFB_ENOMEM = -4,        /* host allocation failed                            */
  MFB_EHIP = -5,          /* a HIP runtime call failed                          */
  MFB_ESTATE = -6         /* handle not ready (e.g. not bound, no potential)   */
} mfb_status;

/* Arithmetic of the sum-factorisation contractions (mfb_apply_H). */
typedef enum {
  MFB_FP64 = 0,       /* float64 on the vector ALUs                            */
  MFB_FP64_MFMA = 1,  /* float64 on the matrix cores (v_mfma_f64_16x16x4f64),
                         float64 accumulation; a measured comparison form      */
  MFB_FP32_MFMA = 2,  /* float32 on the matrix cores, float32 accumulation;
                         quadrature scaling, S and trace stay float64          */
  MFB_FP32 = 3        /* float32 on the vector ALUs (comparison form)          */
} mfb_prec;

/* Operator of mfb_apply_op (eq. fe_matrices). */
typedef enum {
  MFB_OP_H = 0,  /* Hamiltonian: 1/2 grad N_i . grad N_j + N_i V N_j        */
  MFB_OP_M = 1   /* mass matrix: N_i N_j                                     */
} mfb_op;

/* ------------------------------------------------------------------ mesh */

/* Box [0,Lx]x[0,Ly]x[0,Lz] split into nx x ny x nz equal Q_p cells.
 * nx, ny, nz must be even (cells are grouped in 2x2x2 batches, the coarse
 * level of Alg. 1).  degree p in 1..6 (else MFB_EUNSUPPORTED); at p = 5, 6 the
 * applies run the fp64 and fp32 vector forms on box cells (one workgroup
 * per cell), and the matrix-core forms, curved cells and the tuned kernel
 * variants other than 0 and 9 give MFB_EUNSUPPORTED.
 * dirichlet_faces: bit 2d = face x_d = 0, bit 2d+1 = face x_d = L_d.
 * order: 0 = batches along the Hilbert curve (Alg. 1 step 2), 1 = batches
 * in lexicographic order (x fastest).                                      */
typedef struct {
  int32_t nx, ny, nz;
  double Lx, Ly, Lz;
  int32_t degree;
  uint32_t dirichlet_faces;
  int32_t order;
} mfb_mesh_desc;

typedef struct {
  int64_t ndofs;            /* (p nx + 1)(p ny + 1)(p nz + 1) rows            */
  int64_t ncells;
  int32_t nbatches;         /* = number of row blocks                         */
  int32_t degree;
  int32_t qp_per_cell;      /* (p+1)^3                                         */
  int32_t nodes_per_batch;  /* (2p+1)^3                                        */
  size_t meta_bytes;        /* device metadata size for mfb_mesh_bind          */
} mfb_mesh_info;

/* Plans the mesh: batch order (Hilbert, Alg. 1 step 2), first-encounter row
 * numbering and row blocks (Alg. 1 steps 5-7), per-batch gather tables and
 * the 1D basis (Gauss-Lobatto nodes, (p+1)-point Gauss rule).  Host only.
 * Errors: EINVAL (null, non-positive or odd sizes), EUNSUPPORTED (degree). */
int mfb_create_mesh(const mfb_mesh_desc* desc, mfb_mesh** out);
int mfb_mesh_get_info(const mfb_mesh* mesh, mfb_mesh_info* out);

/* Integer coordinates (cx, cy, cz) of every cell in library cell order:
 * cell 8 r + e is child e = ex + 2 ey + 4 ez of the batch in row block r.
 * ijk: host array of ncells*3 int32.                                         */
int mfb_mesh_cells(const mfb_mesh* mesh, int32_t* ijk);

/* Node positions, host array [ndofs][3] in global lexicographic node order
 * (x fastest): the GLL points of every box cell, or the positions given to
 * mfb_mesh_set_nodes.                                                        */
int mfb_mesh_node_points(const mfb_mesh* mesh, double* xyz);

/* Curved cells (Sec. 3.1: general hexahedral meshes).  xyz: host array
 * [ndofs][3] of node positions in global lexicographic node order (x fastest
 * over the index grid of the box).  Each cell becomes the image of the
 * reference cube under the isoparametric Q_p map of its own nodes; the
 * library tabulates, per cell and quadrature point, 1/2 JxW J^{-1} J^{-T}
 * and JxW (JxW = w_q |det J|), and the Hamiltonian and mass operators use
 * them.  Batches, row blocks, supports and the column order stay those of
 * the index grid (the box of the descriptor).  The device layout grows by
 * 56 (p+1)^3 bytes per cell: query mfb_mesh_get_info (meta_bytes) afterwards.
 * Must be called before mfb_mesh_set_potential (ESTATE otherwise).
 * Errors: EINVAL (null, non-finite positions, a singular Jacobian), ESTATE.
 * On curved cells mfb_apply_H_tuned takes the fused kernels (0, 2, 7) only
 * (EUNSUPPORTED otherwise).                                                  */
int mfb_mesh_set_nodes(mfb_mesh* mesh, const double* xyz);

/* Physical quadrature points of every cell, library cell order, q = q1 +
 * n q2 + n^2 q3: host array [ncells][(p+1)^3][3].  On a box x_q = x_K + h (.)
 * xi_q; on curved cells the image of xi_q under the cell's map.              */
int mfb_mesh_qp_points(const mfb_mesh* mesh, double* xyz);

/* Potential values V(x_q) at those points (host array [ncells][(p+1)^3]).
 * The library stores JxW_q V(x_q), the coefficient of the N_i V N_j term of
 * eq. fe_matrices.  Must be called before mfb_mesh_bind.                    */
int mfb_mesh_set_potential(mfb_mesh* mesh, const double* v_qp);

/* Copies the mesh metadata (gather tables, quadrature coefficients) into
 * d_meta (caller-owned device buffer of info.meta_bytes, 256-B aligned).
 * Errors: ESTATE (no potential set), EHIP.                                   */
int mfb_mesh_bind(mfb_mesh* mesh, void* d_meta, void* stream);
void mfb_destroy_mesh(mfb_mesh* mesh);

/* ----------------------------------------------------------- multivector */

/* Sparse multivector layout.  centers: M x 3 orbital centres (original
 * order).  radius: radius_count == 1 (shared) or M values: the patch of an
 * orbital is the set of batches whose centre lies within the radius (the
 * support construction of Sec. 4); block (r, C) is stored iff row block r's
 * batch is in the patch of an orbital of C.  Column blocks: colblock_sizes
 * (ncolblocks values summing to M) or, when NULL, blocks of B with the
 * remainder on the last block (Alg. 2 step 4).  col_order: 0 = Hilbert order
 * of the batch containing each centre (Alg. 2 step 3), 1 = original order.
 * Column blocks wider than 16 are rejected (EUNSUPPORTED).                  */
typedef struct {
  int32_t M;
  const double* centers;
  const double* radius;
  int32_t radius_count;
  int32_t ncolblocks;
  const int32_t* colblock_sizes;
  int32_t B;
  int32_t col_order;
} mfb_mv_desc;

typedef struct {
  int32_t M, nrowblocks, ncolblocks;
  int64_t nblocks;          /* stored blocks                                   */
  int64_t nvalues;          /* float64 values of one multivector (= E)         */
  size_t meta_bytes;        /* device metadata size for mfb_mv_bind            */
  size_t work_bytes;        /* device workspace of mfb_tmmult / tuned apply    */
  int64_t apply_items;      /* (batch, column block, 8-column chunk) items     */
  int64_t apply_pairs;      /* (batch, column block) pairs touching a block    */
  int64_t apply_pairs_own;  /* ... of which the batch's own block is stored    */
  int64_t tm_units;         /* (row block, C1, C2) products of Alg. 8          */
  int64_t s_pairs;          /* stored (C1, C2) blocks of S                     */
  int64_t tm_tasks;         /* densely populated row blocks whose products of
                               Alg. 8 run as one task each (not in tm_units)   */
  int64_t apply_items_own;  /* apply items whose batch's own block is stored
                               (the rest are shell items)                      */
} mfb_mv_info;

/* Table-1-style statistics of a layout (Sec. 4.1, Table 1).                   */
typedef struct {
  double rows_mean, rows_std;        /* row block sizes                        */
  double cols_mean, cols_std;        /* column block sizes                     */
  double blocks_per_row_mean;        /* stored blocks per row block            */
  double colblocks_per_cell_mean;    /* non-empty column blocks per FE cell    */
  double colblocks_per_cell_std;
  int64_t colblocks_per_cell_sum;
} mfb_stats;

int mfb_create_bcsr_multivector(const mfb_mesh* mesh, const mfb_mv_desc* desc, mfb_mv** out);
int mfb_mv_get_info(const mfb_mv* mv, mfb_mv_info* out);
int mfb_query_stats(const mfb_mv* mv, mfb_stats* out);

/* Host views of the pattern (valid while the handle lives):
 * rowptr[nrowblocks+1], colidx[nblocks] (ascending within a row, Sec. 3.4),
 * row_block_start[nrowblocks+1], col_block_start[ncolblocks+1],
 * dof_perm[ndofs] (row -> global node id), col_perm[M] (column -> original
 * orbital), block_offset[nblocks+1], batch_order[nrowblocks] (row block ->
 * batch id bx + nbx (by + nby bz)).                                          */
typedef struct {
  const int64_t* rowptr;
  const int32_t* colidx;
  const int64_t* row_block_start;
  const int32_t* col_block_start;
  const int64_t* dof_perm;
  const int32_t* col_perm;
  const int64_t* block_offset;
  const int32_t* batch_order;
} mfb_pattern_view;
int mfb_mv_pattern(const mfb_mv* mv, mfb_pattern_view* out);

/* Host-side scatter of COO triplets (global node id, original orbital id,
 * value) into a host value array of info.nvalues doubles (entries not named
 * are set to 0).  Errors: EPATTERN when a triplet falls outside the stored
 * blocks (nothing is written then), EINVAL on out-of-range ids.             */
int mfb_mv_pack(const mfb_mv* mv, int64_t nnz, const int64_t* node, const int32_t* orb,
                const double* val, double* values);
/* Coordinates of every stored value position: node[k], orb[k] for
 * k < info.nvalues (host arrays).                                           */
int mfb_mv_entry_coords(const mfb_mv* mv, int64_t* node, int32_t* orb);

/* A second handle with the pattern of x (the destination Y = H X is kept
 * "on the pattern of X", Alg. 6): same rows, columns, stored blocks, value
 * layout and device plan size.  Its own lifetime and binding; calls that take
 * two layouts (mfb_apply_op, mfb_mmult) treat the two as the same pattern.
 * If x is a closure layout the new one is a closure of the same source.
 * Errors: EINVAL (null).                                                    */
int mfb_create_like(const mfb_mv* x, mfb_mv** out);

/* Device bytes of one multivector of this layout (value_bytes = 8 nvalues,
 * the figure an admission rule by BCSR memory footprint needs) and of its
 * device plan (meta_bytes, for mfb_mv_bind).  Host only.  Errors: EINVAL.    */
int mfb_mv_sizes(const mfb_mv* mv, size_t* value_bytes, size_t* meta_bytes);

/* Scatter COO triplets given in global coordinates (host arrays: node id,
 * original orbital id, value) into the device value array d_values
 * (info.nvalues doubles, caller-owned) of layout mv; stored positions not
 * named are set to 0.  Marshalling only: packs on the host, then copies on
 * the stream and waits for the copy.  Errors: EPATTERN when a triplet falls
 * outside the stored blocks and EINVAL on out-of-range ids (d_values is not
 * touched then), EHIP.                                                      */
int mfb_mv_set_global(const mfb_mv* mv, int64_t nnz, const int64_t* node, const int32_t* orb,
                      const double* val, double* d_values, void* stream);

/* The inverse: every stored value of d_values in global coordinates.  val
 * (host, info.nvalues doubles) receives the values in stored order; when
 * node and orb are not NULL (host, info.nvalues each) they receive each
 * position's global node id and original orbital id.  Copies on the stream
 * and waits for the copy.  Errors: EINVAL, EHIP.                            */
int mfb_mv_get_global(const mfb_mv* mv, const double* d_values, int64_t* node, int32_t* orb,
                      double* val, void* stream);

/* Copies the layout's device plan (apply work list, Alg. 8 product list)
 * into d_meta (caller-owned, info.meta_bytes, 256-B aligned).               */
int mfb_mv_bind(mfb_mv* mv, void* d_meta, void* stream);
void mfb_destroy_mv(mfb_mv* mv);

/* --------------------------------------------------------------- compute */

/* Y = mask_P(H X) (Alg. 6: zero the destination, then for every (batch,
 * column block) pair whose batch touches a stored block, gather the batch's
 * node values, integrate with sum factorisation, add into the stored rows).
 * d_X, d_Y: device arrays of info.nvalues doubles in the layout of mv; d_Y
 * is overwritten and must not alias d_X.  Values of X on Dirichlet rows are
 * ignored; Y is 0 there.  Errors: EPATTERN (mv planned on another mesh),
 * ESTATE (mesh or mv not bound), EINVAL (unknown precision), EHIP.           */
int mfb_apply_H(const mfb_mesh* mesh, const mfb_mv* mv, const double* d_X, double* d_Y,
                int prec, void* stream);

/* Y += mask_P(H X): Alg. 6 without its first step (the zero fill), the same
 * kernels otherwise.  With Y zeroed beforehand (mfb_mv_zero) the result is
 * that of mfb_apply_H; the split lets a caller zero the next destination
 * while the current one is in use (two destinations, two streams), so the
 * fill leaves the apply's critical path.  Same arguments and errors as
 * mfb_apply_H; every check happens before anything is enqueued.             */
int mfb_apply_H_acc(const mfb_mesh* mesh, const mfb_mv* mv, const double* d_X, double* d_Y,
                    int prec, void* stream);

/* Y <- 0 on the info.nvalues stored entries of mv's layout (the first step
 * of Alg. 6, as mfb_apply_H runs it).  Errors: EINVAL (null), EHIP.          */
int mfb_mv_zero(const mfb_mv* mv, double* d_Y, void* stream);

/* Same result through an explicitly configured kernel (used by the
 * autotuner).  kernel: even values launch one work unit per workgroup, odd
 * values launch persistent workgroups that pull units from a queue; kernel/2
 * selects how a unit maps onto threads: 0 = the default (currently 1),
 * 1 = a workgroup of 64(p+1) threads per (batch, 8-column chunk) with LDS
 * layout switches, 2 = one wave per unit (p = 2: the whole cell tensor in
 * registers; p = 4: one wave per cell).  Kernels 0 and 2 run own and shell
 * items in one grid; the others check shell items (batches whose own block
 * of C is not stored) in a second kernel.  kernel 6: persistent workgroups
 * of the batch mapping walking a static strided list, with the loads of the
 * next items issued before the current item is computed (no workspace).
 * kernel 7: at p = 2 persistent workgroups of p + 1 compute waves and one
 * loader wave that gathers the next item into a second LDS stage while the
 * current one is computed; at p = 3, 4 on box cells the shared-stage form
 * (one stage, refilled chunk by chunk during the operator), else the fused
 * grid (no workspace).  kernel 8 (p <= 2, vector forms, box cells): one wave
 * per item with each lane's cell tensor in registers.  kernel 9 (p >= 2,
 * vector forms, box cells, no workspace): one workgroup per (item, cell), a
 * thread per (line, column), the operator in five passes over the cell's
 * 8 columns in LDS; mfb_apply_H's kernel at p = 3, 4 in the vector forms
 * (fp64 and fp32) and at p = 5, 6.  At p = 5, 6 only kernels 0 and 9 (both that kernel) are
 * available.
 * grid: for kernels 0 and 2, the shell items checked per wave (a power of
 * two up to 64; 0 = 4 at p <= 2, else 2); for the persistent kernels, the
 * number of workgroups (0 = as many as fit on the device); else unused.  d_work: the workspace (info.work_bytes);
 * it holds the queue counters, so two tuned applies sharing a workspace must
 * not overlap in time.                                                      */
typedef struct {
  int32_t prec;
  int32_t kernel;
  int32_t grid;
  int32_t reserved;
} mfb_tune;
int mfb_apply_H_tuned(const mfb_mesh* mesh, const mfb_mv* mv, const double* d_X, double* d_Y,
                      const mfb_tune* tune, void* d_work, void* stream);

/* Closure destination layout of x, so that the operator's full result can
 * be kept (the result of Alg. 6 has a larger support than its argument):
 * block (r, C) is stored iff a non-Dirichlet node of row block r shares a cell
 * with a non-Dirichlet node whose block (r', C) is stored in x.  H X and M X
 * are zero outside it, so X^T (H X) through mfb_tmmult on this layout is the
 * projected Hamiltonian of eq. energy exactly (symmetric up to rounding).
 * Same rows, columns and column blocks as x; x's stored blocks are a subset.
 * The new layout refers to x: destroy it before x.  It is a destination only
 * (mfb_apply_H, mfb_apply_H_tuned and mfb_mv_update reject it).  Bind it with
 * mfb_mv_bind like any layout (info.meta_bytes); info.work_bytes is the
 * workspace of mfb_tmmult on it.  Errors: EINVAL (closure of a closure),
 * EUNSUPPORTED (2^31 or more stored values).                                */
int mfb_create_closure(const mfb_mv* x, mfb_mv** out);

/* Y = mask_y(op X) with op = H or M (MFB_OP_H / MFB_OP_M, eq. fe_matrices),
 * the same cell loop as mfb_apply_H.  d_X: layout x (info.nvalues of x);
 * d_Y: layout y, which is x itself or a layout created like it (the result
 * is kept on the pattern of X, as mfb_apply_H does) or the closure of x
 * (nothing is dropped).  d_Y is
 * overwritten and must not alias d_X.  prec as for mfb_apply_H; the mass
 * form scales with JxW in float64.  Errors: EPATTERN (y is neither x nor its
 * closure, or another mesh), ESTATE (not bound), EINVAL, EUNSUPPORTED, EHIP. */
int mfb_apply_op(const mfb_mesh* mesh, const mfb_mv* x, const mfb_mv* y, int op,
                 const double* d_X, double* d_Y, int prec, void* stream);

/* Energy of eq. energy, E = tr((2 I - Mbar) Hbar), float64, summed in a
 * fixed order (bitwise repeatable).  d_Mbar, d_Hbar: M x M row-major device
 * arrays (X^T M X and X^T H X, e.g. from mfb_tmmult on a closure layout, in
 * the same column order); d_E: one double; d_work: device scratch of
 * 8 ceil(M/32)^2 bytes (one partial sum per 32x32 tile), 8-byte aligned.
 * Errors: EINVAL, EHIP.                                                     */
int mfb_energy(int32_t M, const double* d_Mbar, const double* d_Hbar, double* d_E, void* d_work,
               void* stream);

/* Alg. 7 with truncation: C = mask_c(A (alpha B + beta I)), or C += that
 * when accumulate != 0.  A lives in layout a, C in layout c; a and c share
 * rows and columns (equal, or one the closure of the other).  Entries of the
 * product outside c's stored blocks are discarded (the destination's pattern
 * decides, as the gradient is denser than X).  d_B: M x M row-major device
 * array in library column order (e.g. Hbar, Mbar from mfb_tmmult), treated
 * as dense.  Each block of C is summed over the blocks of A's row block in a
 * fixed order (bitwise repeatable); d_C must not alias d_A.  With A = M X,
 * H X on the closure and C on X's pattern, two calls give the gradient of
 * eq. gradient: alpha = -2, beta = 0 with B = Hbar, then alpha = -2, beta = 4
 * with B = Mbar, accumulated.  Errors: EPATTERN, ESTATE, EINVAL, EHIP.       */
int mfb_mmult(const mfb_mv* a, const mfb_mv* c, const double* d_A, const double* d_B, double alpha,
              double beta, double* d_C, int accumulate, void* stream);

/* Y += alpha X over the info.nvalues stored values of layout mv (a descent
 * step X <- X - tau G with alpha = -tau).  Errors: EINVAL, EHIP.            */
int mfb_mv_axpy(const mfb_mv* mv, double alpha, const double* d_X, double* d_Y, void* stream);

/* X[:, c] *= scale[c] for every column c (library column order) over the
 * stored values of layout mv, e.g. to normalise columns to X^T M X = 1 on the
 * diagonal.  d_scale: M device doubles.  Errors: EINVAL, ESTATE, EHIP.      */
int mfb_mv_scale_columns(const mfb_mv* mv, const double* d_scale, double* d_X, void* stream);

/* tr(X^T Y) = sum over stored entries of X . Y (eq. G_ops4: the directional
 * derivative tr(D^T G) of a line search), float64, fixed order.  d_out: one
 * double; d_work: 8 KiB of device scratch (1024 partial sums), 8-byte
 * aligned.  Errors: EINVAL, EHIP.                                           */
int mfb_mv_dot(const mfb_mv* mv, const double* d_X, const double* d_Y, double* d_out, void* d_work,
               void* stream);

/* S = X^T Y (Alg. 8) and t = tr S, float64.  X and Y share the layout mv, or
 * mv is a closure layout: then X is in mv's source layout and Y in mv.
 * d_S: M*M doubles, fully written (entries outside the product pattern are
 * exactly 0); d_trace: one double; d_work: info.work_bytes of scratch for the
 * per-row-block partial products, which are summed in a fixed order (the
 * result is bitwise reproducible).  Densely populated row blocks
 * (info.tm_tasks) compute all their block products at once; the partial
 * products and their order of summation are the same.  Errors: ESTATE (not
 * bound), EHIP.                                                              */
int mfb_tmmult(const mfb_mv* mv, const double* d_X, const double* d_Y, double* d_S,
               double* d_trace, void* d_work, void* stream);

/* mfb_tmmult with an explicit shape of its block-product kernels (used by the
 * autotuner, a search over the same computation, Alg. 8): unit_steps and
 * long_steps are the row steps of 8 rows each wave keeps in flight in the
 * products of two 8-wide blocks and in the other products at most 8 wide
 * (4, 8 or 16; 0 = the library's choice, 8 and 4).  The result equals
 * mfb_tmmult's to rounding (the rows are dealt to the waves of a product
 * differently) and is bitwise reproducible for a given shape.  Errors: EINVAL
 * (another step count, null argument, misaligned d_work), ESTATE, EHIP.      */
typedef struct {
  int32_t unit_steps;
  int32_t long_steps;
  int32_t reserved[2];
} mfb_tm_tune;
int mfb_tmmult_tuned(const mfb_mv* mv, const double* d_X, const double* d_Y, double* d_S,
                     double* d_trace, void* d_work, const mfb_tm_tune* tune, void* stream);

/* mfb_tmmult without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory: code under HIP graph capture,
 * serving loops that must not call hipMalloc, harnesses that forbid it.  The
 * per-row-block partial products go to a fixed array of 64 MiB in device
 * memory (67108864 bytes, one per GPU, kept until the process ends); a
 * layout whose info.work_bytes exceed it is refused with EINVAL before
 * anything is enqueued (use mfb_tmmult with a workspace then).  Results are
 * those of mfb_tmmult (the same kernels, the same order of summation).  The
 * array is shared by every call on a GPU and keeps the last call's partial
 * products; nothing in it needs clearing (every slot a call reads is
 * written by the same call first), but calls that overlap in time on one GPU
 * (different streams) race on it and give wrong results: serialise them.
 * The stream must belong to the current device.  Errors: EINVAL, ESTATE,
 * EHIP.                                                                      */
int mfb_tmmult_noalloc(const mfb_mv* mv, const double* d_X, const double* d_Y, double* d_S,
                       double* d_trace, void* stream);

/* Column-scaled update on the stored entries of X, the iteration of the
 * serving loop: X <- X - tau (Y - X diag(S) / diag(S2)), where column c of X
 * is scaled by S[c][c] / S2[c][c] (0 when S2[c][c] == 0).  S and S2 are M x M
 * as written by mfb_tmmult (for instance S = X^T Y and S2 = X^T X), so each
 * column moves along its own residual Y_c - X_c (X_c.Y_c / X_c.X_c)
 * (eq. G_ops4 supplies the column-wise inner products).  The pattern of X is
 * kept.  Errors: ESTATE (not bound), EHIP.                                  */
int mfb_mv_update(const mfb_mv* mv, double* d_X, const double* d_Y, const double* d_S,
                  const double* d_S2, double tau, void* stream);

/* Measurement instrument: the fp64 vector-ALU rate this device reaches, the
 * roof the vector forms of the apply are held against (Sec. 4.2 compares its
 * kernels' GFlop/s with the machine's).  Launches `blocks` workgroups of 256
 * threads; each thread runs 16 independent chains of `iters` fused
 * multiply-adds (32 iters flops).  d_out: at least 8 bytes of device memory,
 * written only if the chains reach a value they cannot reach (it keeps the
 * arithmetic from being removed).  The caller times the launch on its stream
 * (flops = blocks * 256 * 32 * iters).  Errors: EINVAL (blocks or iters < 1,
 * null d_out), EHIP.                                                         */
int mfb_probe_fp64_fma(double* d_out, int64_t blocks, int32_t iters, void* stream);

/* Thread-local message describing the last error (empty if none).           */
const char* mfb_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MFBCSR_H */
