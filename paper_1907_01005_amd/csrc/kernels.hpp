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
  const ApplyItem* items;
  int64_t nitems;
  const int32_t* gtab;   // [rank][ (2p+1)^3 ]
  const double* cV;      // [cell 8 rank + e][ (p+1)^3 ]
  int32_t* counters;     // 8 queue counters (persistent kernel only)
  int32_t grid;          // persistent workgroups
  int32_t pad;
  double S[25];          // S[q*n + k] = phi_k(xq_q)
  double Dco[25];        // collocation derivative on the Gauss points
  double W2[25];         // W2[a*n + b] = w_a w_b
  double w[5];           // 1D Gauss weights
  double cg[3];          // 1/2 hx hy hz / h_d^2
};

struct TmParams {
  const double* X;
  const double* Y;
  const TmUnit* units;
  int64_t nunits;
  double* part;
  const int32_t* pair_tab;   // [ncb*ncb]
  const int32_t* pair_ptr;   // [npairs+1]
  const int64_t* pair_list;
  const int32_t* cb_of_col;  // [M]
  const int32_t* cb_start;   // [ncb+1]
  int32_t M, ncb;
  double* S;
  double* trace;
};

// prec: 0 fp64 VALU, 1 fp64 MFMA, 2 fp32 MFMA, 3 fp32 VALU.
// kernel: 0 one item per workgroup, 1 persistent queue.
// Returns a hipError_t value (0 on success) or -2 for an unsupported variant.
int launch_apply(const ApplyParams& p, int degree, int prec, int kernel, int64_t nvalues,
                 void* stream);
int launch_tmmult(const TmParams& p, void* stream);
int device_cu_count();

}  // namespace gpu
}  // namespace mfb
