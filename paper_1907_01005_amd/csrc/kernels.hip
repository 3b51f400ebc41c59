// Device kernels for gfx950: matrix-free Hamiltonian on BCSR multivectors
// (Alg. 6 of the paper) and the block overlap product S = X^T Y (Alg. 8).
//
// Apply: one work item = one 8-column chunk of a column block C on one
// 2x2x2 batch of cells.  A workgroup of 64 (p+1) threads handles an item:
// thread t works on column t%8 of cell (t/8)%8 and owns one plane of the
// cell's (p+1)^3 tensor.  In "layout A" the plane is z = const (the thread
// holds the x-y slice), in "layout B" it is y = const (x-z slice).  The
// contractions along x run in either layout, along y in A and along z in B;
// switching layouts goes through one LDS tile per cell-column.  The cell
// operator is the sum-factorised form of eq. fe_matrices:
//
//   u_q = (S x S x S) u,   g_d = c_d (.) D_d u_q,   v = c_V (.) u_q,
//   out = (S^T x S^T x S^T) ( v + sum_d D_d^T g_d )
//
// with S the 1D interpolation to the Gauss points, D the collocation
// derivative on the Gauss points, c_d = 1/2 JxW / h_d^2 and c_V = JxW V.
// The eight cell results are summed per batch node in LDS (fixed order)
// and added to Y with float64 atomics on the rows whose block is stored.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.hpp"

namespace mfb {
namespace gpu {
int device_cu_count();
namespace {

// -------------------------------------------------------------- helpers
// out[o0][o1] = sum_k M(o_AX, k) in[...k...]; M(o,k) = M[o*n+k], or M[k*n+o]
// when TR (the transposed matrix).  AX = index of `in` that is contracted.
template <int n, int AX, bool TR, typename R>
__device__ __forceinline__ void contract(const R* __restrict__ M, const R (&in)[n][n],
                                         R (&out)[n][n]) {
#pragma unroll
  for (int o0 = 0; o0 < n; ++o0)
#pragma unroll
    for (int o1 = 0; o1 < n; ++o1) {
      const int o = AX == 0 ? o0 : o1;
      R s = 0;
#pragma unroll
      for (int k = 0; k < n; ++k) {
        const R c = TR ? M[k * n + o] : M[o * n + k];
        const R x = AX == 0 ? in[k][o1] : in[o0][k];
        s = __builtin_fma(c, x, s);
      }
      out[o0][o1] = s;
    }
}

template <int n, int AX, bool TR, typename R>
__device__ __forceinline__ void contract_add(const R* __restrict__ M, const R (&in)[n][n],
                                             R (&acc)[n][n]) {
#pragma unroll
  for (int o0 = 0; o0 < n; ++o0)
#pragma unroll
    for (int o1 = 0; o1 < n; ++o1) {
      const int o = AX == 0 ? o0 : o1;
      R s = acc[o0][o1];
#pragma unroll
      for (int k = 0; k < n; ++k) {
        const R c = TR ? M[k * n + o] : M[o * n + k];
        const R x = AX == 0 ? in[k][o1] : in[o0][k];
        s = __builtin_fma(c, x, s);
      }
      acc[o0][o1] = s;
    }
}

// Workgroup index -> item index so that each XCD (workgroups are dealt to
// the 8 XCDs round robin) walks one contiguous, Hilbert-ordered range.
__device__ __forceinline__ int64_t xcd_item(int64_t wg, int64_t nwg) {
  const int64_t per = nwg >> 3;  // nwg is a multiple of 8
  return (wg & 7) * per + (wg >> 3);
}

// -------------------------------------------------------------- apply
template <typename R, int P>
struct Shape {
  static constexpr int n = P + 1, n2 = n * n, n3 = n2 * n;
  static constexpr int NB = 2 * P + 1, NB3 = NB * NB * NB;
  static constexpr int NT = 64 * n;  // threads per workgroup
};

template <typename R, int P>
__device__ __forceinline__ void apply_item(const ApplyParams& a, const ApplyItem* __restrict__ it,
                                           R* __restrict__ T, int64_t* __restrict__ s_off) {
  using Sh = Shape<R, P>;
  constexpr int n = Sh::n, n2 = Sh::n2, n3 = Sh::n3, NB = Sh::NB, NB3 = Sh::NB3, NT = Sh::NT;
  const int t = threadIdx.x;
  const int c = t & 7, e = (t >> 3) & 7, pl = t >> 6;
  const int ex = e & 1, ey = (e >> 1) & 1, ez = e >> 2;
  const int cc = t & 63;  // cell-column slot of this thread

  if (t < 27) s_off[t] = it->off[t];
  const int rank = it->rank, c0 = it->c0, nc = it->nc, ld = it->ld;
  __syncthreads();

  R Sm[n * n], Dm[n * n];
#pragma unroll
  for (int i = 0; i < n * n; ++i) {
    Sm[i] = (R)a.S[i];
    Dm[i] = (R)a.Dco[i];
  }
  const int32_t* __restrict__ g = a.gtab + (int64_t)rank * NB3;

  // gather the z = pl plane of this cell-column (layout A)
  R u[n][n];
  bool any = false;
#pragma unroll
  for (int j = 0; j < n; ++j)
#pragma unroll
    for (int i = 0; i < n; ++i) {
      const int v = (ex * P + i) + NB * ((ey * P + j) + NB * (ez * P + pl));
      const int32_t ent = g[v];
      double x = 0.0;
      if (c < nc && ent >= 0) {
        const int64_t off = s_off[ent >> 24];
        if (off >= 0) x = a.X[off + (int64_t)(ent & 0xFFFFFF) * ld + c0 + c];
      }
      u[i][j] = (R)x;
      any |= (x != 0.0);
    }
  // an item whose gathered values are all zero contributes exactly zero
  if (!__syncthreads_or(any)) return;

  R* __restrict__ Tc = T + cc * n3;
  R A[n][n], B[n][n];
  // forward interpolation along x and y (layout A)
  contract<n, 0, false>(Sm, u, A);
  contract<n, 1, false>(Sm, A, B);
#pragma unroll
  for (int j = 0; j < n; ++j)
#pragma unroll
    for (int i = 0; i < n; ++i) Tc[i + n * j + n2 * pl] = B[i][j];
  __syncthreads();
  // layout B: plane y = pl (already at its Gauss point)
#pragma unroll
  for (int k = 0; k < n; ++k)
#pragma unroll
    for (int i = 0; i < n; ++i) A[i][k] = Tc[i + n * pl + n2 * k];
  R uq[n][n];
  contract<n, 1, false>(Sm, A, uq);  // along z: uq[x][z] at y = pl
  const double wpl = a.w[pl];
  const double sx = a.cg[0] * wpl, sy = a.cg[1] * wpl, sz = a.cg[2] * wpl;
  R wB[n][n];
  // x-gradient
  contract<n, 0, false>(Dm, uq, A);
#pragma unroll
  for (int i = 0; i < n; ++i)
#pragma unroll
    for (int k = 0; k < n; ++k) A[i][k] = (R)((double)A[i][k] * (sx * a.W2[i * n + k]));
  contract<n, 0, true>(Dm, A, wB);
  // z-gradient
  contract<n, 1, false>(Dm, uq, A);
#pragma unroll
  for (int i = 0; i < n; ++i)
#pragma unroll
    for (int k = 0; k < n; ++k) A[i][k] = (R)((double)A[i][k] * (sz * a.W2[i * n + k]));
  contract_add<n, 1, true>(Dm, A, wB);
  // potential term, float64: c_V = JxW V
  {
    const double* __restrict__ cv = a.cV + ((int64_t)rank * 8 + e) * n3 + n * pl;
#pragma unroll
    for (int i = 0; i < n; ++i)
#pragma unroll
      for (int k = 0; k < n; ++k)
        wB[i][k] = (R)((double)wB[i][k] + cv[i + n2 * k] * (double)uq[i][k]);
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < n; ++k)
#pragma unroll
    for (int i = 0; i < n; ++i) Tc[i + n * pl + n2 * k] = uq[i][k];
  __syncthreads();
  // layout A again (plane z = pl): y-gradient
#pragma unroll
  for (int j = 0; j < n; ++j)
#pragma unroll
    for (int i = 0; i < n; ++i) A[i][j] = Tc[i + n * j + n2 * pl];
  contract<n, 1, false>(Dm, A, B);
#pragma unroll
  for (int i = 0; i < n; ++i)
#pragma unroll
    for (int j = 0; j < n; ++j) B[i][j] = (R)((double)B[i][j] * (sy * a.W2[i * n + j]));
  contract<n, 1, true>(Dm, B, A);  // A = D_y^T g_y   (layout A)
  __syncthreads();
#pragma unroll
  for (int j = 0; j < n; ++j)
#pragma unroll
    for (int i = 0; i < n; ++i) Tc[i + n * j + n2 * pl] = A[i][j];
  __syncthreads();
  // layout B: add the y part, then integrate back along z
#pragma unroll
  for (int k = 0; k < n; ++k)
#pragma unroll
    for (int i = 0; i < n; ++i) wB[i][k] += Tc[i + n * pl + n2 * k];
  contract<n, 1, true>(Sm, wB, A);  // A[x][z nodal] at y = pl (Gauss)
  __syncthreads();
#pragma unroll
  for (int k = 0; k < n; ++k)
#pragma unroll
    for (int i = 0; i < n; ++i) Tc[i + n * pl + n2 * k] = A[i][k];
  __syncthreads();
  // layout A: integrate back along y and x
#pragma unroll
  for (int j = 0; j < n; ++j)
#pragma unroll
    for (int i = 0; i < n; ++i) A[i][j] = Tc[i + n * j + n2 * pl];
  contract<n, 1, true>(Sm, A, B);
  contract<n, 0, true>(Sm, B, A);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < n; ++j)
#pragma unroll
    for (int i = 0; i < n; ++i) Tc[i + n * j + n2 * pl] = A[i][j];
  __syncthreads();

  // sum the cell results per batch node and add into the stored rows of Y
  for (int idx = t; idx < NB3 * 8; idx += NT) {
    const int col = idx & 7, v = idx >> 3;
    if (col >= nc) continue;
    const int32_t ent = g[v];
    if (ent < 0) continue;
    const int64_t off = s_off[ent >> 24];
    if (off < 0) continue;
    const int vx = v % NB, vy = (v / NB) % NB, vz = v / (NB * NB);
    double acc = 0.0;
#pragma unroll
    for (int sz2 = 0; sz2 < 2; ++sz2) {
      const int lz = vz - sz2 * P;
      if (lz < 0 || lz > P) continue;
#pragma unroll
      for (int sy2 = 0; sy2 < 2; ++sy2) {
        const int ly = vy - sy2 * P;
        if (ly < 0 || ly > P) continue;
#pragma unroll
        for (int sx2 = 0; sx2 < 2; ++sx2) {
          const int lx = vx - sx2 * P;
          if (lx < 0 || lx > P) continue;
          const int ce = sx2 + 2 * sy2 + 4 * sz2;
          acc += (double)T[(ce * 8 + col) * n3 + lx + n * ly + n2 * lz];
        }
      }
    }
    unsafeAtomicAdd(a.Y + off + (int64_t)(ent & 0xFFFFFF) * ld + c0 + col, acc);
  }
}

template <typename R, int P>
__global__ __launch_bounds__(64 * (P + 1)) void apply_grid_kernel(ApplyParams a) {
  using Sh = Shape<R, P>;
  __shared__ R T[64 * Sh::n3];
  __shared__ int64_t s_off[27];
  const int64_t item = xcd_item(blockIdx.x, gridDim.x);
  if (item >= a.nitems) return;
  apply_item<R, P>(a, a.items + item, T, s_off);
}

// Persistent form: each workgroup pulls items from the queue of its XCD's
// contiguous range, then from the other XCDs' ranges.  Every counter only
// grows, so every workgroup leaves once all eight ranges are exhausted.
template <typename R, int P>
__global__ __launch_bounds__(64 * (P + 1)) void apply_queue_kernel(ApplyParams a) {
  using Sh = Shape<R, P>;
  __shared__ R T[64 * Sh::n3];
  __shared__ int64_t s_off[27];
  __shared__ int64_t s_item;
  const int64_t per = (a.nitems + 7) >> 3;
  const int home = blockIdx.x & 7;
  for (int q = 0; q < 8; ++q) {
    const int xcd = (home + q) & 7;
    const int64_t lo = xcd * per;
    const int64_t hi = min(a.nitems, lo + per);
    while (true) {
      __syncthreads();
      if (threadIdx.x == 0) {
        const int64_t k = atomicAdd(a.counters + xcd, 1);
        s_item = lo + k;
      }
      __syncthreads();
      const int64_t item = s_item;
      if (item >= hi) break;
      apply_item<R, P>(a, a.items + item, T, s_off);
    }
  }
}

// -------------------------------------------------------------- utilities
__global__ void fill_zero_kernel(double* __restrict__ p, int64_t n, int32_t* counters) {
  if (counters && blockIdx.x == 0 && threadIdx.x < 8) counters[threadIdx.x] = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t n2 = n >> 1;
  double2* p2 = reinterpret_cast<double2*>(p);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += stride)
    p2[i] = make_double2(0.0, 0.0);
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) p[n - 1] = 0.0;
}

// -------------------------------------------------------------- overlap
// Stage 1: one wave per block product X_{r,C1}^T Y_{r,C2}.  Lane (s, a)
// walks rows s, s+R, ... of the row block (R = 64 / |C1|) and keeps the
// |C2| products of column a; the R partial rows are summed in LDS in a
// fixed order.
constexpr int kTmWaves = 4;
__global__ __launch_bounds__(64 * kTmWaves) void tm_stage1_kernel(TmParams p) {
  __shared__ double red[kTmWaves][64][17];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t u = (int64_t)blockIdx.x * kTmWaves + wv;
  const bool valid = u < p.nunits;
  TmUnit U;
  if (valid) U = p.units[u];
  else U = TmUnit{0, 0, 0, 0, 1, 1, 0};
  const int w1 = U.w1, w2 = U.w2;
  const int R = 64 / w1;
  const int s = lane / w1, col = lane - s * w1;
  double acc[16];
#pragma unroll
  for (int b = 0; b < 16; ++b) acc[b] = 0.0;
  if (valid && s < R) {
    const double* __restrict__ X = p.X + U.off1;
    const double* __restrict__ Y = p.Y + U.off2;
    for (int i = s; i < U.rows; i += R) {
      const double x = X[(int64_t)i * w1 + col];
      const double* __restrict__ y = Y + (int64_t)i * w2;
#pragma unroll
      for (int b = 0; b < 16; ++b)
        if (b < w2) acc[b] = __builtin_fma(x, y[b], acc[b]);
    }
  }
#pragma unroll
  for (int b = 0; b < 16; ++b) red[wv][lane][b] = acc[b];
  __syncthreads();
  if (valid) {
    for (int idx = lane; idx < w1 * w2; idx += 64) {
      const int aa = idx / w2, bb = idx - aa * w2;
      double sum = 0.0;
      for (int g = 0; g < R; ++g) sum += red[wv][g * w1 + aa][bb];
      p.part[U.part + idx] = sum;
    }
  }
}

// Stage 2: every entry of S sums the partial products of its block pair in
// row-block order; entries outside the product pattern are set to zero.
__global__ __launch_bounds__(256) void tm_stage2_kernel(TmParams p) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t MM = (int64_t)p.M * p.M;
  if (e >= MM) return;
  const int al = (int)(e / p.M), be = (int)(e - (int64_t)al * p.M);
  const int C1 = p.cb_of_col[al], C2 = p.cb_of_col[be];
  const int pid = p.pair_tab[(int64_t)C1 * p.ncb + C2];
  double sum = 0.0;
  if (pid >= 0) {
    const int a = al - p.cb_start[C1], b = be - p.cb_start[C2];
    const int w2 = p.cb_start[C2 + 1] - p.cb_start[C2];
    const int at = a * w2 + b;
    for (int k = p.pair_ptr[pid]; k < p.pair_ptr[pid + 1]; ++k) sum += p.part[p.pair_list[k] + at];
  }
  p.S[e] = sum;
}

// Stage 3: trace of S with a fixed-shape tree reduction.
__global__ __launch_bounds__(256) void tm_trace_kernel(TmParams p) {
  __shared__ double red[256];
  double s = 0.0;
  for (int al = threadIdx.x; al < p.M; al += 256) s += p.S[(int64_t)al * p.M + al];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *p.trace = red[0];
}

template <typename R, int P>
hipError_t launch_apply_t(const ApplyParams& p, int kernel, hipStream_t st) {
  using Sh = Shape<R, P>;
  if (p.nitems == 0) return hipSuccess;
  if (kernel == 0) {
    const int64_t nwg = ((p.nitems + 7) / 8) * 8;
    hipLaunchKernelGGL((apply_grid_kernel<R, P>), dim3((unsigned)nwg), dim3(Sh::NT), 0, st, p);
  } else {
    int grid = p.grid;
    if (grid <= 0) {
      int per_cu = 0;
      hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void*>(&apply_queue_kernel<R, P>), Sh::NT, 0);
      if (e != hipSuccess) return e;
      grid = std::max(1, per_cu) * std::max(1, device_cu_count());
    }
    hipLaunchKernelGGL((apply_queue_kernel<R, P>), dim3((unsigned)grid), dim3(Sh::NT), 0, st, p);
  }
  return hipGetLastError();
}

}  // namespace

int device_cu_count() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return cus;
}

int launch_apply(const ApplyParams& p, int degree, int prec, int kernel, int64_t nvalues,
                 void* stream) {
  hipStream_t st = (hipStream_t)stream;
  {
    const int64_t blocks = std::min<int64_t>(4096, std::max<int64_t>(1, (nvalues / 2 + 255) / 256));
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p.Y, nvalues,
                       kernel == 1 ? p.counters : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
  }
  hipError_t e;
  if (prec == 0) {
    e = degree == 2 ? launch_apply_t<double, 2>(p, kernel, st) : launch_apply_t<double, 4>(p, kernel, st);
  } else if (prec == 3) {
    e = degree == 2 ? launch_apply_t<float, 2>(p, kernel, st) : launch_apply_t<float, 4>(p, kernel, st);
  } else {
    return -2;
  }
  return (int)e;
}

int launch_tmmult(const TmParams& p, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (p.nunits > 0) {
    const int64_t g1 = (p.nunits + kTmWaves - 1) / kTmWaves;
    hipLaunchKernelGGL(tm_stage1_kernel, dim3((unsigned)g1), dim3(64 * kTmWaves), 0, st, p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
  }
  const int64_t MM = (int64_t)p.M * p.M;
  hipLaunchKernelGGL(tm_stage2_kernel, dim3((unsigned)((MM + 255) / 256)), dim3(256), 0, st, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return (int)e;
  hipLaunchKernelGGL(tm_trace_kernel, dim3(1), dim3(256), 0, st, p);
  return (int)hipGetLastError();
}

}  // namespace gpu
}  // namespace mfb
