// Host-side planning of the mesh and of BCSR multivector layouts.
//
// Nothing here touches the GPU: the structures built here are copied to
// device memory by the bind calls and read by the kernels in kernels.hip.
#pragma once

#include <array>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace mfb {

// Error carrying an mfb_status code; converted at the C boundary.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

// ---------------------------------------------------------------- 1D basis
// Lagrange polynomials on p+1 Gauss-Lobatto-Legendre nodes of [0,1] and the
// (p+1)-point Gauss-Legendre rule (Sec. 3.1: Lagrange shape functions,
// continuous across cells).
struct Basis1D {
  int p = 0, n = 0;
  std::vector<double> nodes;  // n GLL nodes, ascending
  std::vector<double> xq, wq; // n Gauss points (ascending) and weights
  std::vector<double> S;      // S[q*n + k] = phi_k(xq[q])
  std::vector<double> Dco;    // Dco[q*n + j] = psi_j'(xq[q]); psi = Lagrange basis on the Gauss points
};
Basis1D make_basis(int p);

// Hilbert index of an integer point of a 2^bits cube (Skilling's transform).
uint64_t hilbert3(uint32_t x, uint32_t y, uint32_t z, int bits);
int bits_for(int extent);

// ---------------------------------------------------------------- mesh
constexpr int kMaxDeg = 6;

struct MeshPlan {
  int nc[3] = {0, 0, 0};   // cells per axis
  int p = 0, n = 0, NB = 0; // degree, p+1, 2p+1
  double L[3] = {0, 0, 0}, h[3] = {0, 0, 0};
  unsigned dirichlet = 0;
  int order = 0;
  int nb[3] = {0, 0, 0};   // batches per axis
  int nbatch = 0;
  int64_t na[3] = {0, 0, 0}; // nodes per axis
  int64_t N = 0, ncells = 0;
  std::vector<int32_t> batch_order;  // rank -> batch id
  std::vector<int32_t> batch_rank;   // batch id -> rank
  std::vector<int64_t> rb_start;     // nbatch + 1
  std::vector<int64_t> dof_perm;     // row -> node
  std::vector<int64_t> node_row;     // node -> row
  std::vector<int32_t> node_rb;      // node -> row block
  std::vector<uint8_t> is_dirichlet; // node -> 0/1
  // per rank: NB^3 entries, (slot << 24) | row-in-owner-block, or -1 (Dirichlet)
  std::vector<int32_t> gtab;
  Basis1D basis;
  std::vector<double> cV;            // [cell 8r+e][q]: JxW_q V(x_q)
  bool has_potential = false;
  // curved cells (node positions given): the isoparametric map of each cell
  bool curved = false;
  std::vector<double> nodes;         // [N][3] node positions, global lexicographic order
  std::vector<double> cG;            // [cell 8r+e][6][q]: 1/2 JxW (J^{-1} J^{-T}) 00,11,22,01,02,12
  std::vector<double> cJ;            // [cell 8r+e][q]: JxW_q = w_q |det J(q)|

  int64_t node_id(int64_t X, int64_t Y, int64_t Z) const { return X + na[0] * (Y + na[1] * Z); }
  void batch_coords(int b, int& bx, int& by, int& bz) const {
    bx = b % nb[0]; by = (b / nb[0]) % nb[1]; bz = b / (nb[0] * nb[1]);
  }
};

void plan_mesh(MeshPlan& m, const int nc[3], const double L[3], int degree, unsigned dirichlet,
               int order);
void mesh_cells(const MeshPlan& m, int32_t* ijk);
void mesh_qp_points(const MeshPlan& m, double* xyz);
// Positions of the box's nodes (GLL points inside each cell), [N][3], global
// lexicographic order; the positions given to mesh_set_nodes on curved cells.
void mesh_node_points(const MeshPlan& m, double* xyz);
void mesh_set_potential(MeshPlan& m, const double* v);
// Curved cells: node positions [N][3] define every cell's isoparametric map
// (Sec. 3.1: general hexahedral cells).  Fills nodes, cG and cJ; throws on a
// singular Jacobian.  Must come before mesh_set_potential.
void mesh_set_nodes(MeshPlan& m, const double* xyz);

// ---------------------------------------------------------------- layouts
// One work item of the apply kernel: an 8-column chunk of column block C on
// the 2x2x2 cells of the batch with rank `rank`.  off[s] is the value offset
// of block (owner row block of neighbour slot s, C), or -1 when that block
// is not stored (or slot s owns no node of this batch).
struct ApplyItem {
  int32_t rank;
  int32_t c0;   // first column of the chunk within C
  int32_t nc;   // columns in the chunk (1..8)
  int32_t ld;   // |C|: row stride of the blocks of C
  int64_t off[27];
};
static_assert(sizeof(ApplyItem) == 232, "ApplyItem layout");

// One block product of Alg. 8: X_{r,C1}^T Y_{r,C2} into partial[part].
// tslot >= 0 for the products with C1 = C2: the slot of its own trace
// (sum over the block's diagonal) in the overlap's diagonal list.
struct TmUnit {
  int64_t off1, off2, part;
  int32_t rows, w1, w2, tslot;
};
static_assert(sizeof(TmUnit) == 40, "TmUnit layout");

// One block of S for the second overlap stage: its pair's n partial
// products start at part[base] (n = 0: the block is outside the pattern).
struct S2Desc {
  int64_t base;
  int32_t n, c1, c2, w1, w2, pad;
};
static_assert(sizeof(S2Desc) == 32, "S2Desc layout");

// A run of densely populated row blocks of Alg. 8 as one task: every
// product X_{r,C1}^T Y_{r,C2} of its row blocks at once, over the union of
// their column blocks (ka on the X side, kb on the Y side), X and Y read
// once.  Segment s covers task rows [seg_start[s], seg_start[s + 1]), row
// block r0 + s.  The blocks of segment s are task_blk[a_first + s ka + i]
// (X side) and task_blk[b_first + s kb + j] (Y side), offset -1 where that
// row block does not store the block.  The partial of union pair (i, j) goes
// to task_part[p_first + i kb + j], -1 where the pair meets in no member.
constexpr int kTaskMaxSeg = 4;
struct TmTask {
  int64_t a_first, b_first, p_first;
  int32_t rows, ka, kb, wa, wb, nseg;
  int32_t seg_start[kTaskMaxSeg + 1];
  int32_t pad;
};
static_assert(sizeof(TmTask) == 72, "TmTask layout");
struct TaskBlk {
  int64_t off;  // value offset of the block, -1 if not stored in this segment
  int32_t col;  // first column within the task's columns
  int32_t w;    // block width
};
static_assert(sizeof(TaskBlk) == 16, "TaskBlk layout");

struct MvPlan {
  const MeshPlan* mesh = nullptr;
  int M = 0, ncb = 0;
  std::vector<int32_t> col_perm;     // column -> original orbital
  std::vector<int32_t> col_pos;      // original orbital -> column
  std::vector<int32_t> cb_start;     // ncb + 1
  std::vector<int32_t> cb_of_col;    // column -> column block
  std::vector<int64_t> rowptr;       // nbatch + 1
  std::vector<int32_t> colidx;
  std::vector<int64_t> block_offset; // nblocks + 1
  std::vector<ApplyItem> items;      // own items (batch's own block stored) then shell items
  std::vector<int32_t> item_cb;      // column block of each item (host only)
  int64_t n_own_items = 0;
  std::vector<int32_t> rowoff;       // [item][(2p+1)^3] value offset of each node's row at the item's first column, or -1
  std::vector<int32_t> shell_ptr;    // [nshell+1] CSR over the shell items' present rows
  std::vector<int32_t> shell_ro;     // present row offsets of the shell items
  int64_t apply_pairs = 0, apply_pairs_own = 0;
  std::vector<TmUnit> units;         // Alg. 8 block products, sorted by kernel class:
  // 0: 8x8 blocks of at most 128 rows, 1: other blocks at most 8 wide on
  // both sides, 2: wider blocks of at most 128 rows, 3: the rest
  std::array<int64_t, 4> tm_class_end{};  // cumulative unit counts per class
  std::vector<TmTask> tasks;         // dense row blocks, by tile class (widths <= 64, 96, 128)
  std::array<int64_t, 3> task_class_end{};
  std::vector<TaskBlk> task_blk;
  std::vector<int64_t> task_part;
  std::vector<S2Desc> s2;            // [ncb*ncb] blocks of S, most partials first
  int64_t part_doubles = 0;
  int64_t ndiag = 0;                 // units with C1 = C2 (one trace slot each)
  std::vector<int32_t> pair_tab;     // ncb*ncb -> pair id or -1
  std::vector<int32_t> pair_ptr;     // npairs + 1: prefix count of partial products per pair
  std::vector<int64_t> pair_list;    // npairs: offset of the pair's contiguous partials
  // closure layouts only: the layout whose operator results this one holds,
  // and for every apply item of that layout the offset of each batch node's
  // row here (at the item's first column), or -1
  const MvPlan* source = nullptr;
  std::vector<int32_t> dest_rowoff;
  // cell statistics
  std::vector<int32_t> cell_colblocks; // per library cell: non-empty column blocks
  int64_t block_index(int r, int C) const;  // -1 if (r, C) not stored
};

void plan_mv(MvPlan& mv, const MeshPlan& m, int M, const double* centers, const double* radius,
             int radius_count, int ncolblocks, const int32_t* sizes, int B, int col_order);

// Row blocks with at least kTaskMinPairs and at most kTaskMaxPairs block
// pairs, no more than kTaskMaxWidth columns on either side and at most
// kTaskMaxRows rows qualify for tasks.  A task walks its rows in a chain of
// 16-row chunks, so longer row blocks stay with the units, which spread
// their rows over the lanes.  Runs of qualifying row blocks are merged while
// the union stays within the pair limit, kTaskMaxRunRows rows and the width
// class (64, 96, 128 columns) of its widest member, and its products cost at
// most kTaskMaxWaste times the members' own.
constexpr int kTaskMinPairs = 16;
constexpr int kTaskMaxPairs = 512;
constexpr int kTaskMaxWidth = 128;
constexpr int kTaskMaxRows = 128;
constexpr int kTaskMaxRunRows = 160;
constexpr double kTaskMaxWaste = 1.25;

// Overlap plan (units, tasks, pairs, S-block descriptors) of S = A^T B into mv.
void plan_overlap(MvPlan& mv, const MvPlan& A, const MvPlan& B, const MeshPlan& m);

// Closure destination of x: block (r, C) is stored iff a non-Dirichlet node of
// row block r shares a cell with a non-Dirichlet node whose block (r', C) is
// stored in x, so H X and M X lie in it entirely.  Same rows and columns as
// x; x's stored blocks are a subset.  Also plans the destination row offsets
// of x's apply items and the overlap X^T Y (X in x, Y here).  No apply items
// of its own: a closure layout is a destination only.
void plan_closure(MvPlan& y, const MvPlan& x, const MeshPlan& m);

}  // namespace mfb
