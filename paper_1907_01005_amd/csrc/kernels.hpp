// Host-side view of the device kernels (launchers live in kernels.hip).
#pragma once

#include <cstdint>

#include "planner.hpp"

namespace mfb {
namespace gpu {

// Kernel arguments of the apply kernels.  The 1D tables are passed by value
// so that every workgroup reads them from the kernel-argument segment.
struct ApplyParams {
  const double* X;
  double* Y;
  const ApplyItem* items;   // items whose batch's own block is stored
  int64_t nitems;
  const ApplyItem* shell;   // items of batches whose own block is not stored
  int64_t nshell;
  const int32_t* rowoff;    // [own items, shell items][(2p+1)^3]: offset of each node's row at the item's first column, or -1
  const int32_t* shell_ptr; // [nshell+1] CSR over the present rows of the shell items
  const int32_t* shell_ro;  // present row offsets
  const int32_t* gtab;   // [rank][ (2p+1)^3 ]
  const double* cV;      // [cell 8 rank + e][ (p+1)^3 ]
  int32_t* counters;     // 8 queue counters (persistent kernel only)
  int32_t grid;          // persistent workgroups, or shell items per wave (fused grid)
  int32_t pad;
  // 1D tables, n = p + 1 <= 7 (the kernels of p <= 4 read the first n^2)
  double S[49];          // S[q*n + k] = phi_k(xq_q)
  double Dco[25];        // collocation derivative on the Gauss points (p <= 4)
  float Sf[49];          // float copies of S and Dco for the float contractions
  float Df[25];
  const double* Wg;      // [3][ (p+1)^3 ]: 1/2 JxW_q / h_d^2 per direction d
  const double* jxw;     // [ (p+1)^3 ]: JxW_q (mass operator)
  const int32_t* rowoff_out;  // destination offsets per item and node (rowoff, or a closure's)
  // curved cells only (else null): per cell 8 rank + e, the metric
  // 1/2 JxW J^{-1} J^{-T} as six planes [00, 11, 22, 01, 02, 12][ (p+1)^3 ]
  // and JxW [ (p+1)^3 ]
  const double* cG;
  const double* cJ;
  // box cells, register-resident kernel: Dw[o*n + k] = w_o Dco[o*n + k] (w the
  // Gauss weights), and per direction d the scale of each line along d,
  // gline[d][a + n b] = 1/2 hx hy hz / h_d^2 w_a w_b with (a, b) the indices
  // of the line along the other two axes in increasing axis order
  double Dw[25];
  float Dwf[25];
  double gline[3][25];
  // the 1D stiffness K1 = D^T diag(w) D on the Gauss points (symmetric, and
  // unchanged under (o, k) -> (n-1-o, n-1-k))
  double K1[49];
  float K1f[49];
  // the line scales as factors (p >= 5): gline[d][a + n b] = gfac[d] wq[a] wq[b]
  double wq[8];
  double gfac[3];        // 1/2 hx hy hz / h_d^2
  int64_t nvalues_x;     // stored values of X (the extent of d_X)
};

struct TmParams {
  const double* X;
  const double* Y;
  const TmUnit* units;
  int64_t nunits;
  int64_t class_end[4];      // cumulative unit counts of the four stage-1 kernel classes
  const TmTask* tasks;       // dense row blocks, sorted by width class
  const TaskBlk* task_blk;
  const int64_t* task_part;
  int64_t task_class_end[3]; // cumulative task counts (widths <= 64, 96, 128)
  double* part;
  const int32_t* pair_tab;   // [ncb*ncb]
  const int32_t* pair_ptr;   // [npairs+1] prefix counts of partial products per pair
  const int64_t* pair_list;  // [npairs] offset of each pair's contiguous partials
  const int32_t* cb_of_col;  // [M]
  const int32_t* cb_start;   // [ncb+1]
  const S2Desc* s2;          // [ncb*ncb] blocks of S for the second stage
  int64_t max_pair_parts;    // most partial products of one pair
  double* tdiag;             // [ndiag] traces of the products with C1 = C2
  int64_t ndiag;
  int32_t fold_trace;        // 1: the trace is summed from tdiag in the second stage
  int32_t M, ncb;
  double* S;
  double* trace;
};

// prec: 0 fp64 VALU, 1 fp64 MFMA, 2 fp32 MFMA, 3 fp32 VALU.
// kernel: -1 the library's choice (mfb_apply_H), 0/1 default processor as
// grid/queue, 2/3 batch processor, 4/5 single-wave processor
// (register-resident for p = 2, per cell for p = 4), 6 pipelined persistent,
// 7 loader pipeline, 8 register-resident waves.
// Returns a hipError_t value (0 on success) or -2 for an unsupported variant.
int launch_apply(const ApplyParams& p, int degree, int prec, int kernel, int64_t nvalues,
                 void* stream, bool fill = true);
// Y[0 .. n) = 0 with the apply's fill kernel.
int launch_zero(double* Y, int64_t n, void* stream);
// unit_steps, long_steps: row steps of 8 rows in flight per wave in the two
// block-product classes (4, 8 or 16; 0 = the defaults, 8 and 4).
int launch_tmmult(const TmParams& p, void* stream, int unit_steps = 0, int long_steps = 0);
// Fixed device scratch of the allocation-free overlap: kScratchBytes per GPU;
// scratch_address gives this device's address (a hipError_t value on failure).
constexpr size_t kScratchBytes = size_t(64) << 20;
int scratch_address(void** out);
// kernel 8 (register-resident waves): p <= 2, vector-ALU contractions
// (fp64 or fp32), box cells.
bool reg_kernel_supported(int degree, int prec, bool curved);
// op: 0 Hamiltonian, 1 mass; default kernel; destination nvalues for the fill.
int launch_apply_op(const ApplyParams& p, int degree, int prec, int op, int64_t nvalues,
                    void* stream);
int launch_energy(int M, const double* Mbar, const double* Hbar, double* E, double* work,
                  void* stream);

// X <- X - tau (Y - X d), d_c = S[c][c] / S2[c][c], one workgroup per stored block.
struct UpdateParams {
  double* X;
  const double* Y;
  const double* S;
  const double* S2;
  const int64_t* blk_off;   // [nblocks+1] value offsets
  const int32_t* blk_col0;  // [nblocks] first column of the block's column block
  const int32_t* blk_w;     // [nblocks] width of the column block
  int64_t nblocks;
  int32_t M;
  double tau;
};
int launch_update(const UpdateParams& p, void* stream);

// Device view of a layout's stored blocks (CSR over row blocks).
struct BlockView {
  const int64_t* rowptr;    // [nrowblocks+1]
  const int64_t* blk_off;   // [nblocks+1] value offset of each block
  const int32_t* blk_col0;  // [nblocks] first column of the block's column block
  const int32_t* blk_w;     // [nblocks] its width
  const int32_t* blk_row;   // [nblocks] its row block
  int64_t nblocks;
};

// Alg. 7: C = [C +] mask_c(A (alpha B + beta I)), B dense M x M row-major.
struct MmultParams {
  const double* A;
  const double* B;
  double* C;
  BlockView a, c;
  int32_t M;
  int32_t accumulate;
  double alpha, beta;
  int64_t max_rows;         // largest row block of c (picks the kernel shape)
};
int launch_mmult(const MmultParams& p, void* stream);
int launch_axpy(int64_t n, double alpha, const double* X, double* Y, void* stream);
int launch_scale_columns(const BlockView& v, const double* scale, double* X, void* stream);
// fixed-order dot product; work: kDotPartials doubles
constexpr int kDotPartials = 1024;
int launch_dot(int64_t n, const double* X, const double* Y, double* out, double* work, void* stream);
int device_cu_count();
// fp64 fused multiply-add rate probe: blocks x 256 threads, 16 chains of
// iters FMAs each; out written only on an impossible value.
int launch_probe_fma(double* out, int64_t blocks, int32_t iters, void* stream);

}  // namespace gpu
}  // namespace mfb
