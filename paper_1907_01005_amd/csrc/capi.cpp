// The C boundary of the library (include/mfbcsr.h).  Every entry point
// converts exceptions into status codes and keeps a thread-local message.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "mfbcsr.h"
#include "kernels.hpp"
#include "planner.hpp"

namespace {

thread_local std::string g_err;
std::atomic<uint64_t> g_next_pattern_id{1};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct MeshLayout {
  size_t off_gtab = 0, off_cv = 0, off_wg = 0, off_cg = 0, off_cj = 0, bytes = 0;
};

MeshLayout mesh_layout(const mfb::MeshPlan& m) {
  MeshLayout L;
  const size_t nb3 = (size_t)m.NB * m.NB * m.NB, n3 = (size_t)m.n * m.n * m.n;
  L.off_gtab = 0;
  L.off_cv = align256(sizeof(int32_t) * nb3 * m.nbatch);
  L.off_wg = align256(L.off_cv + sizeof(double) * (size_t)m.ncells * n3);
  L.bytes = align256(L.off_wg + sizeof(double) * 4 * n3);
  if (m.curved) {  // the metric (six planes) and JxW of every cell
    L.off_cg = L.bytes;
    L.off_cj = align256(L.off_cg + sizeof(double) * (size_t)m.ncells * 6 * n3);
    L.bytes = align256(L.off_cj + sizeof(double) * (size_t)m.ncells * n3);
  }
  return L;
}

// Per-direction quadrature scaling of the gradient term of eq. fe_matrices on
// a box cell, 1/2 JxW_q / h_d^2 with JxW_q = w_q1 w_q2 w_q3 hx hy hz, for
// d = 0, 1, 2; then JxW_q itself (the mass term).
std::vector<double> grad_scales(const mfb::MeshPlan& m) {
  const int n = m.n, n3 = n * n * n;
  const double det = m.h[0] * m.h[1] * m.h[2];
  std::vector<double> wg(4 * n3);
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        const double jxw = m.basis.wq[i] * m.basis.wq[j] * m.basis.wq[k] * det;
        for (int d = 0; d < 3; ++d) wg[d * n3 + i + n * (j + n * k)] = 0.5 * jxw / (m.h[d] * m.h[d]);
        wg[3 * n3 + i + n * (j + n * k)] = jxw;
      }
  return wg;
}

struct MvLayout {
  size_t off_items = 0, off_units = 0, off_pair_tab = 0, off_pair_ptr = 0, off_pair_list = 0,
         off_cb_of_col = 0, off_cb_start = 0, off_blk_off = 0, off_blk_col0 = 0, off_blk_w = 0,
         off_rowoff = 0, off_shell_ptr = 0, off_shell_ro = 0, off_s2 = 0, off_dest_rowoff = 0,
         off_rowptr = 0, off_blk_row = 0, off_tasks = 0, off_task_blk = 0, off_task_part = 0,
         bytes = 0;
};

MvLayout mv_layout(const mfb::MvPlan& v) {
  MvLayout L;
  size_t o = 0;
  L.off_items = o;
  o = align256(o + sizeof(mfb::ApplyItem) * v.items.size());
  L.off_units = o;
  o = align256(o + sizeof(mfb::TmUnit) * v.units.size());
  L.off_pair_tab = o;
  o = align256(o + sizeof(int32_t) * v.pair_tab.size());
  L.off_pair_ptr = o;
  o = align256(o + sizeof(int32_t) * v.pair_ptr.size());
  L.off_pair_list = o;
  o = align256(o + sizeof(int64_t) * v.pair_list.size());
  L.off_cb_of_col = o;
  o = align256(o + sizeof(int32_t) * v.cb_of_col.size());
  L.off_cb_start = o;
  o = align256(o + sizeof(int32_t) * v.cb_start.size());
  L.off_blk_off = o;
  o = align256(o + sizeof(int64_t) * v.block_offset.size());
  L.off_blk_col0 = o;
  o = align256(o + sizeof(int32_t) * v.colidx.size());
  L.off_blk_w = o;
  o = align256(o + sizeof(int32_t) * v.colidx.size());
  L.off_rowoff = o;
  o = align256(o + sizeof(int32_t) * v.rowoff.size());
  L.off_shell_ptr = o;
  o = align256(o + sizeof(int32_t) * v.shell_ptr.size());
  L.off_shell_ro = o;
  o = align256(o + sizeof(int32_t) * v.shell_ro.size());
  L.off_s2 = o;
  o = align256(o + sizeof(mfb::S2Desc) * v.s2.size());
  L.off_dest_rowoff = o;
  o = align256(o + sizeof(int32_t) * v.dest_rowoff.size());
  L.off_rowptr = o;
  o = align256(o + sizeof(int64_t) * v.rowptr.size());
  L.off_blk_row = o;
  o = align256(o + sizeof(int32_t) * v.colidx.size());
  L.off_tasks = o;
  o = align256(o + sizeof(mfb::TmTask) * v.tasks.size());
  L.off_task_blk = o;
  o = align256(o + sizeof(mfb::TaskBlk) * v.task_blk.size());
  L.off_task_part = o;
  o = align256(o + sizeof(int64_t) * v.task_part.size());

  L.bytes = std::max<size_t>(o, 256);
  return L;
}

constexpr size_t kCounterBytes = 256;  // queue counters at the head of the workspace

void fail(int code, const std::string& msg) { throw mfb::Error(code, msg); }

void check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(MFB_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

struct mfb_mesh {
  mfb::MeshPlan plan;
  MeshLayout lay;
  void* d_meta = nullptr;
  bool bound = false;
};

struct mfb_mv {
  mfb::MvPlan plan;
  const mfb_mesh* mesh = nullptr;
  const mfb_mv* source = nullptr;  // closure layouts: the layout they are the closure of
  uint64_t pattern_id = 0;         // equal for a layout and the layouts created like it
  MvLayout lay;
  size_t work_bytes = 0;
  void* d_meta = nullptr;
  bool bound = false;
  std::vector<int64_t> rowptr_view;
};

#define MFB_TRY try {
#define MFB_CATCH                                   \
  }                                                 \
  catch (const mfb::Error& e) {                     \
    g_err = e.what();                               \
    return e.code;                                  \
  }                                                 \
  catch (const std::bad_alloc&) {                   \
    g_err = "host allocation failed";               \
    return MFB_ENOMEM;                              \
  }                                                 \
  catch (const std::exception& e) {                 \
    g_err = e.what();                               \
    return MFB_EINVAL;                              \
  }                                                 \
  catch (...) {                                     \
    g_err = "unknown error";                        \
    return MFB_EINVAL;                              \
  }

extern "C" {

const char* mfb_last_error(void) { return g_err.c_str(); }

int mfb_create_mesh(const mfb_mesh_desc* desc, mfb_mesh** out) {
  MFB_TRY
  if (!desc || !out) fail(MFB_EINVAL, "null argument");
  *out = nullptr;
  auto* m = new mfb_mesh();
  try {
    const int nc[3] = {desc->nx, desc->ny, desc->nz};
    const double L[3] = {desc->Lx, desc->Ly, desc->Lz};
    mfb::plan_mesh(m->plan, nc, L, desc->degree, desc->dirichlet_faces, desc->order);
    m->lay = mesh_layout(m->plan);
  } catch (...) {
    delete m;
    throw;
  }
  *out = m;
  return MFB_OK;
  MFB_CATCH
}

int mfb_mesh_get_info(const mfb_mesh* mesh, mfb_mesh_info* out) {
  MFB_TRY
  if (!mesh || !out) fail(MFB_EINVAL, "null argument");
  const auto& m = mesh->plan;
  out->ndofs = m.N;
  out->ncells = m.ncells;
  out->nbatches = m.nbatch;
  out->degree = m.p;
  out->qp_per_cell = m.n * m.n * m.n;
  out->nodes_per_batch = m.NB * m.NB * m.NB;
  out->meta_bytes = mesh->lay.bytes;
  return MFB_OK;
  MFB_CATCH
}

int mfb_mesh_cells(const mfb_mesh* mesh, int32_t* ijk) {
  MFB_TRY
  if (!mesh || !ijk) fail(MFB_EINVAL, "null argument");
  mfb::mesh_cells(mesh->plan, ijk);
  return MFB_OK;
  MFB_CATCH
}

int mfb_mesh_qp_points(const mfb_mesh* mesh, double* xyz) {
  MFB_TRY
  if (!mesh || !xyz) fail(MFB_EINVAL, "null argument");
  mfb::mesh_qp_points(mesh->plan, xyz);
  return MFB_OK;
  MFB_CATCH
}

int mfb_mesh_node_points(const mfb_mesh* mesh, double* xyz) {
  MFB_TRY
  if (!mesh || !xyz) fail(MFB_EINVAL, "null argument");
  mfb::mesh_node_points(mesh->plan, xyz);
  return MFB_OK;
  MFB_CATCH
}

int mfb_mesh_set_nodes(mfb_mesh* mesh, const double* xyz) {
  MFB_TRY
  if (!mesh || !xyz) fail(MFB_EINVAL, "null argument");
  if (mesh->plan.has_potential) fail(MFB_ESTATE, "set the node positions before the potential");
  for (int64_t i = 0; i < 3 * mesh->plan.N; ++i)
    if (!std::isfinite(xyz[i])) fail(MFB_EINVAL, "node positions must be finite");
  mfb::mesh_set_nodes(mesh->plan, xyz);
  mesh->lay = mesh_layout(mesh->plan);
  mesh->bound = false;
  return MFB_OK;
  MFB_CATCH
}

int mfb_mesh_set_potential(mfb_mesh* mesh, const double* v_qp) {
  MFB_TRY
  if (!mesh || !v_qp) fail(MFB_EINVAL, "null argument");
  mfb::mesh_set_potential(mesh->plan, v_qp);
  mesh->bound = false;
  return MFB_OK;
  MFB_CATCH
}

int mfb_mesh_bind(mfb_mesh* mesh, void* d_meta, void* stream) {
  MFB_TRY
  if (!mesh || !d_meta) fail(MFB_EINVAL, "null argument");
  if (((uintptr_t)d_meta & 255) != 0) fail(MFB_EINVAL, "d_meta must be 256-byte aligned");
  const auto& m = mesh->plan;
  if (!m.has_potential) fail(MFB_ESTATE, "set the potential before binding the mesh");
  std::vector<char> host(mesh->lay.bytes, 0);
  std::memcpy(host.data() + mesh->lay.off_gtab, m.gtab.data(), sizeof(int32_t) * m.gtab.size());
  std::memcpy(host.data() + mesh->lay.off_cv, m.cV.data(), sizeof(double) * m.cV.size());
  const std::vector<double> wg = grad_scales(m);
  std::memcpy(host.data() + mesh->lay.off_wg, wg.data(), sizeof(double) * wg.size());
  if (m.curved) {
    std::memcpy(host.data() + mesh->lay.off_cg, m.cG.data(), sizeof(double) * m.cG.size());
    std::memcpy(host.data() + mesh->lay.off_cj, m.cJ.data(), sizeof(double) * m.cJ.size());
  }
  hipStream_t st = (hipStream_t)stream;
  check_hip(hipMemcpyAsync(d_meta, host.data(), host.size(), hipMemcpyHostToDevice, st),
            "hipMemcpyAsync(mesh metadata)");
  check_hip(hipStreamSynchronize(st), "hipStreamSynchronize");
  mesh->d_meta = d_meta;
  mesh->bound = true;
  return MFB_OK;
  MFB_CATCH
}

void mfb_destroy_mesh(mfb_mesh* mesh) { delete mesh; }

int mfb_create_bcsr_multivector(const mfb_mesh* mesh, const mfb_mv_desc* desc, mfb_mv** out) {
  MFB_TRY
  if (!mesh || !desc || !out) fail(MFB_EINVAL, "null argument");
  *out = nullptr;
  auto* v = new mfb_mv();
  try {
    mfb::plan_mv(v->plan, mesh->plan, desc->M, desc->centers, desc->radius, desc->radius_count,
                 desc->ncolblocks, desc->colblock_sizes, desc->B, desc->col_order);
    v->mesh = mesh;
    v->lay = mv_layout(v->plan);
    v->work_bytes = kCounterBytes + sizeof(double) * (size_t)(v->plan.part_doubles + v->plan.ndiag);
    v->pattern_id = g_next_pattern_id++;
  } catch (...) {
    delete v;
    throw;
  }
  *out = v;
  return MFB_OK;
  MFB_CATCH
}

int mfb_mv_get_info(const mfb_mv* mv, mfb_mv_info* out) {
  MFB_TRY
  if (!mv || !out) fail(MFB_EINVAL, "null argument");
  const auto& p = mv->plan;
  out->M = p.M;
  out->nrowblocks = mv->mesh->plan.nbatch;
  out->ncolblocks = p.ncb;
  out->nblocks = (int64_t)p.colidx.size();
  out->nvalues = p.block_offset.back();
  out->meta_bytes = mv->lay.bytes;
  out->work_bytes = mv->work_bytes;
  out->apply_items = (int64_t)p.items.size();
  out->apply_items_own = p.n_own_items;
  out->apply_pairs = p.apply_pairs;
  out->apply_pairs_own = p.apply_pairs_own;
  out->tm_units = (int64_t)p.units.size();
  out->s_pairs = (int64_t)p.pair_ptr.size() - 1;
  out->tm_tasks = (int64_t)p.tasks.size();
  return MFB_OK;
  MFB_CATCH
}

int mfb_query_stats(const mfb_mv* mv, mfb_stats* out) {
  MFB_TRY
  if (!mv || !out) fail(MFB_EINVAL, "null argument");
  const auto& p = mv->plan;
  const auto& m = mv->mesh->plan;
  auto meanstd = [](const std::vector<double>& x, double& mu, double& sd) {
    double s = 0, s2 = 0;
    for (double v : x) s += v;
    mu = x.empty() ? 0.0 : s / x.size();
    for (double v : x) s2 += (v - mu) * (v - mu);
    sd = x.empty() ? 0.0 : std::sqrt(s2 / x.size());
  };
  std::vector<double> rows(m.nbatch), cols(p.ncb), cells(m.ncells);
  for (int r = 0; r < m.nbatch; ++r) rows[r] = (double)(m.rb_start[r + 1] - m.rb_start[r]);
  for (int C = 0; C < p.ncb; ++C) cols[C] = p.cb_start[C + 1] - p.cb_start[C];
  int64_t sum = 0;
  for (int64_t c = 0; c < m.ncells && !p.cell_colblocks.empty(); ++c) {
    cells[c] = p.cell_colblocks[c];
    sum += p.cell_colblocks[c];
  }
  meanstd(rows, out->rows_mean, out->rows_std);
  meanstd(cols, out->cols_mean, out->cols_std);
  meanstd(cells, out->colblocks_per_cell_mean, out->colblocks_per_cell_std);
  out->colblocks_per_cell_sum = sum;
  out->blocks_per_row_mean = (double)p.colidx.size() / m.nbatch;
  return MFB_OK;
  MFB_CATCH
}

int mfb_mv_pattern(const mfb_mv* mv, mfb_pattern_view* out) {
  MFB_TRY
  if (!mv || !out) fail(MFB_EINVAL, "null argument");
  const auto& p = mv->plan;
  const auto& m = mv->mesh->plan;
  out->rowptr = p.rowptr.data();
  out->colidx = p.colidx.data();
  out->row_block_start = m.rb_start.data();
  out->col_block_start = p.cb_start.data();
  out->dof_perm = m.dof_perm.data();
  out->col_perm = p.col_perm.data();
  out->block_offset = p.block_offset.data();
  out->batch_order = m.batch_order.data();
  return MFB_OK;
  MFB_CATCH
}

int mfb_mv_pack(const mfb_mv* mv, int64_t nnz, const int64_t* node, const int32_t* orb,
                const double* val, double* values) {
  MFB_TRY
  if (!mv || !values || (nnz > 0 && (!node || !orb || !val))) fail(MFB_EINVAL, "null argument");
  if (nnz < 0) fail(MFB_EINVAL, "negative count");
  const auto& p = mv->plan;
  const auto& m = mv->mesh->plan;
  std::vector<int64_t> pos(nnz);
  for (int64_t k = 0; k < nnz; ++k) {
    if (node[k] < 0 || node[k] >= m.N) fail(MFB_EINVAL, "node id out of range");
    if (orb[k] < 0 || orb[k] >= p.M) fail(MFB_EINVAL, "orbital id out of range");
    const int r = m.node_rb[node[k]];
    const int col = p.col_pos[orb[k]];
    const int C = p.cb_of_col[col];
    const int64_t b = p.block_index(r, C);
    if (b < 0) fail(MFB_EPATTERN, "entry outside the stored blocks");
    const int64_t w = p.cb_start[C + 1] - p.cb_start[C];
    pos[k] = p.block_offset[b] + (m.node_row[node[k]] - m.rb_start[r]) * w + (col - p.cb_start[C]);
  }
  std::memset(values, 0, sizeof(double) * (size_t)p.block_offset.back());
  for (int64_t k = 0; k < nnz; ++k) values[pos[k]] = val[k];
  return MFB_OK;
  MFB_CATCH
}

int mfb_mv_entry_coords(const mfb_mv* mv, int64_t* node, int32_t* orb) {
  MFB_TRY
  if (!mv || !node || !orb) fail(MFB_EINVAL, "null argument");
  const auto& p = mv->plan;
  const auto& m = mv->mesh->plan;
  for (int r = 0; r < m.nbatch; ++r) {
    const int64_t r0 = m.rb_start[r], rows = m.rb_start[r + 1] - r0;
    for (int64_t k = p.rowptr[r]; k < p.rowptr[r + 1]; ++k) {
      const int C = p.colidx[k];
      const int c0 = p.cb_start[C], w = p.cb_start[C + 1] - c0;
      int64_t o = p.block_offset[k];
      for (int64_t i = 0; i < rows; ++i)
        for (int j = 0; j < w; ++j, ++o) {
          node[o] = m.dof_perm[r0 + i];
          orb[o] = p.col_perm[c0 + j];
        }
    }
  }
  return MFB_OK;
  MFB_CATCH
}

int mfb_create_like(const mfb_mv* x, mfb_mv** out) {
  MFB_TRY
  if (!x || !out) fail(MFB_EINVAL, "null argument");
  *out = nullptr;
  auto* v = new mfb_mv();
  try {
    v->plan = x->plan;
    v->mesh = x->mesh;
    v->source = x->source;
    v->pattern_id = x->pattern_id;
    v->lay = x->lay;
    v->work_bytes = x->work_bytes;
  } catch (...) {
    delete v;
    throw;
  }
  *out = v;
  return MFB_OK;
  MFB_CATCH
}

int mfb_mv_sizes(const mfb_mv* mv, size_t* value_bytes, size_t* meta_bytes) {
  MFB_TRY
  if (!mv || !value_bytes || !meta_bytes) fail(MFB_EINVAL, "null argument");
  *value_bytes = sizeof(double) * (size_t)mv->plan.block_offset.back();
  *meta_bytes = mv->lay.bytes;
  return MFB_OK;
  MFB_CATCH
}

int mfb_mv_set_global(const mfb_mv* mv, int64_t nnz, const int64_t* node, const int32_t* orb,
                      const double* val, double* d_values, void* stream) {
  MFB_TRY
  if (!mv || !d_values) fail(MFB_EINVAL, "null argument");
  std::vector<double> host((size_t)std::max<int64_t>(1, mv->plan.block_offset.back()));
  const int rc = mfb_mv_pack(mv, nnz, node, orb, val, host.data());
  if (rc != MFB_OK) return rc;
  const size_t bytes = sizeof(double) * (size_t)mv->plan.block_offset.back();
  hipStream_t st = (hipStream_t)stream;
  if (bytes) {
    check_hip(hipMemcpyAsync(d_values, host.data(), bytes, hipMemcpyHostToDevice, st),
              "hipMemcpyAsync(values)");
    check_hip(hipStreamSynchronize(st), "hipStreamSynchronize");
  }
  return MFB_OK;
  MFB_CATCH
}

int mfb_mv_get_global(const mfb_mv* mv, const double* d_values, int64_t* node, int32_t* orb,
                      double* val, void* stream) {
  MFB_TRY
  if (!mv || !d_values || !val) fail(MFB_EINVAL, "null argument");
  if ((node == nullptr) != (orb == nullptr)) fail(MFB_EINVAL, "give both node and orb, or neither");
  const size_t bytes = sizeof(double) * (size_t)mv->plan.block_offset.back();
  hipStream_t st = (hipStream_t)stream;
  if (bytes) {
    check_hip(hipMemcpyAsync(val, d_values, bytes, hipMemcpyDeviceToHost, st),
              "hipMemcpyAsync(values)");
    check_hip(hipStreamSynchronize(st), "hipStreamSynchronize");
  }
  if (node) {
    const int rc = mfb_mv_entry_coords(mv, node, orb);
    if (rc != MFB_OK) return rc;
  }
  return MFB_OK;
  MFB_CATCH
}

int mfb_mv_bind(mfb_mv* mv, void* d_meta, void* stream) {
  MFB_TRY
  if (!mv || !d_meta) fail(MFB_EINVAL, "null argument");
  if (((uintptr_t)d_meta & 255) != 0) fail(MFB_EINVAL, "d_meta must be 256-byte aligned");
  const auto& p = mv->plan;
  const auto& L = mv->lay;
  std::vector<char> host(L.bytes, 0);
  auto put = [&](size_t off, const void* src, size_t n) {
    if (n) std::memcpy(host.data() + off, src, n);
  };
  put(L.off_items, p.items.data(), sizeof(mfb::ApplyItem) * p.items.size());
  put(L.off_units, p.units.data(), sizeof(mfb::TmUnit) * p.units.size());
  put(L.off_pair_tab, p.pair_tab.data(), sizeof(int32_t) * p.pair_tab.size());
  put(L.off_pair_ptr, p.pair_ptr.data(), sizeof(int32_t) * p.pair_ptr.size());
  put(L.off_pair_list, p.pair_list.data(), sizeof(int64_t) * p.pair_list.size());
  put(L.off_cb_of_col, p.cb_of_col.data(), sizeof(int32_t) * p.cb_of_col.size());
  put(L.off_cb_start, p.cb_start.data(), sizeof(int32_t) * p.cb_start.size());
  put(L.off_blk_off, p.block_offset.data(), sizeof(int64_t) * p.block_offset.size());
  put(L.off_rowoff, p.rowoff.data(), sizeof(int32_t) * p.rowoff.size());
  put(L.off_shell_ptr, p.shell_ptr.data(), sizeof(int32_t) * p.shell_ptr.size());
  put(L.off_shell_ro, p.shell_ro.data(), sizeof(int32_t) * p.shell_ro.size());
  put(L.off_s2, p.s2.data(), sizeof(mfb::S2Desc) * p.s2.size());
  put(L.off_dest_rowoff, p.dest_rowoff.data(), sizeof(int32_t) * p.dest_rowoff.size());
  put(L.off_rowptr, p.rowptr.data(), sizeof(int64_t) * p.rowptr.size());
  put(L.off_tasks, p.tasks.data(), sizeof(mfb::TmTask) * p.tasks.size());
  put(L.off_task_blk, p.task_blk.data(), sizeof(mfb::TaskBlk) * p.task_blk.size());
  put(L.off_task_part, p.task_part.data(), sizeof(int64_t) * p.task_part.size());
  {
    std::vector<int32_t> brow(p.colidx.size());
    for (size_t r = 0; r + 1 < p.rowptr.size(); ++r)
      for (int64_t k = p.rowptr[r]; k < p.rowptr[r + 1]; ++k) brow[k] = (int32_t)r;
    put(L.off_blk_row, brow.data(), sizeof(int32_t) * brow.size());
  }

  {
    std::vector<int32_t> col0(p.colidx.size()), wid(p.colidx.size());
    for (size_t k = 0; k < p.colidx.size(); ++k) {
      col0[k] = p.cb_start[p.colidx[k]];
      wid[k] = p.cb_start[p.colidx[k] + 1] - p.cb_start[p.colidx[k]];
    }
    put(L.off_blk_col0, col0.data(), sizeof(int32_t) * col0.size());
    put(L.off_blk_w, wid.data(), sizeof(int32_t) * wid.size());
  }
  hipStream_t st = (hipStream_t)stream;
  check_hip(hipMemcpyAsync(d_meta, host.data(), host.size(), hipMemcpyHostToDevice, st),
            "hipMemcpyAsync(layout metadata)");
  check_hip(hipStreamSynchronize(st), "hipStreamSynchronize");
  mv->d_meta = d_meta;
  mv->bound = true;
  return MFB_OK;
  MFB_CATCH
}

void mfb_destroy_mv(mfb_mv* mv) { delete mv; }

static void fill_apply_params(const mfb_mesh* mesh, const mfb_mv* mv, const double* X, double* Y,
                              mfb::gpu::ApplyParams& a) {
  const auto& m = mesh->plan;
  const auto& b = m.basis;
  std::memset(&a, 0, sizeof(a));
  a.X = X;
  a.Y = Y;
  a.nvalues_x = mv->plan.block_offset.back();
  const char* mb = (const char*)mv->d_meta;
  const char* gb = (const char*)mesh->d_meta;
  a.items = (const mfb::ApplyItem*)(mb + mv->lay.off_items);
  a.nitems = mv->plan.n_own_items;
  a.shell = a.items + mv->plan.n_own_items;
  a.nshell = (int64_t)mv->plan.items.size() - mv->plan.n_own_items;
  a.rowoff = (const int32_t*)(mb + mv->lay.off_rowoff);
  a.shell_ptr = (const int32_t*)(mb + mv->lay.off_shell_ptr);
  a.shell_ro = (const int32_t*)(mb + mv->lay.off_shell_ro);
  a.gtab = (const int32_t*)(gb + mesh->lay.off_gtab);
  a.cV = (const double*)(gb + mesh->lay.off_cv);
  a.Wg = (const double*)(gb + mesh->lay.off_wg);
  a.jxw = a.Wg + 3 * m.n * m.n * m.n;
  a.rowoff_out = a.rowoff;
  a.cG = m.curved ? (const double*)(gb + mesh->lay.off_cg) : nullptr;
  a.cJ = m.curved ? (const double*)(gb + mesh->lay.off_cj) : nullptr;
  const int n = m.n;
  for (int i = 0; i < n * n; ++i) {
    a.S[i] = b.S[i];
    a.Sf[i] = (float)b.S[i];
  }
  if (n <= 5) {
    for (int i = 0; i < n * n; ++i) {
      a.Dco[i] = b.Dco[i];
      a.Df[i] = (float)b.Dco[i];
      a.Dw[i] = b.wq[i / n] * b.Dco[i];
      a.Dwf[i] = (float)a.Dw[i];
    }
  }
  for (int i = 0; i < n; ++i) a.wq[i] = b.wq[i];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double k1 = 0.0;
      for (int q = 0; q < n; ++q) k1 += b.Dco[q * n + i] * b.wq[q] * b.Dco[q * n + j];
      a.K1[i * n + j] = k1;
      a.K1f[i * n + j] = (float)k1;
    }
  const double det = m.h[0] * m.h[1] * m.h[2];
  for (int d = 0; d < 3; ++d) {
    a.gfac[d] = 0.5 * det / (m.h[d] * m.h[d]);
    if (n <= 5)
      for (int q = 0; q < n * n; ++q) a.gline[d][q] = a.gfac[d] * b.wq[q % n] * b.wq[q / n];
  }
}

// The same BCSR pattern: one handle, or layouts created like one another.
static bool same_pattern(const mfb_mv* a, const mfb_mv* b) {
  return a == b || (a->pattern_id != 0 && a->pattern_id == b->pattern_id);
}

static void check_apply_args(const mfb_mesh* mesh, const mfb_mv* mv, const double* X, const double* Y) {
  if (!mesh || !mv || !X || !Y) fail(MFB_EINVAL, "null argument");
  if (mv->mesh != mesh) fail(MFB_EPATTERN, "layout was planned on another mesh");
  if (mv->source) fail(MFB_EINVAL, "a closure layout is a destination only");
  if (!mesh->bound) fail(MFB_ESTATE, "mesh metadata not bound");
  if (!mv->bound) fail(MFB_ESTATE, "layout metadata not bound");
  if (X == Y) fail(MFB_EINVAL, "X and Y must not alias");
}

// Alg. 6 with (fill) or without its zero fill.
static void apply_H_impl(const mfb_mesh* mesh, const mfb_mv* mv, const double* d_X, double* d_Y,
                         int prec, void* stream, bool fill) {
  check_apply_args(mesh, mv, d_X, d_Y);
  if (prec < 0 || prec > 3) fail(MFB_EINVAL, "unknown precision");
  mfb::gpu::ApplyParams a;
  fill_apply_params(mesh, mv, d_X, d_Y, a);
  // the library's choice (-1) for the fp64 and matrix-core forms: at p = 2 the
  // loader pipeline, or the fused grid when there are few items per CU (fp64);
  // at p >= 3 on box cells the line kernel (fp64) or the shared-stage pipeline
  // (matrix cores: 97.6 against 109.0 us for fp64-MFMA with the fused grid on
  // the 64x40x40 box at p = 2, 159 against 186 on the 32x20x20 box at p = 4);
  // the fused grid on curved cells.  The fp32 VALU form: the line kernel (9)
  // at p >= 3 on box cells (60 against 73 us for the fused grid at p = 4),
  // else the fused grid (0).
  int kernel = prec == MFB_FP32 ? 0 : -1;
  if (prec == MFB_FP32 && mesh->plan.p >= 3 && !mesh->plan.curved) kernel = 9;
  const int rc = mfb::gpu::launch_apply(a, mesh->plan.p, prec, kernel, mv->plan.block_offset.back(),
                                        stream, fill);
  if (rc == -2) fail(MFB_EUNSUPPORTED, "precision not implemented by the library");
  if (rc != 0) fail(MFB_EHIP, std::string("kernel launch: ") + hipGetErrorString((hipError_t)rc));
}

int mfb_apply_H(const mfb_mesh* mesh, const mfb_mv* mv, const double* d_X, double* d_Y, int prec,
                void* stream) {
  MFB_TRY
  apply_H_impl(mesh, mv, d_X, d_Y, prec, stream, true);
  return MFB_OK;
  MFB_CATCH
}

int mfb_apply_H_acc(const mfb_mesh* mesh, const mfb_mv* mv, const double* d_X, double* d_Y,
                    int prec, void* stream) {
  MFB_TRY
  apply_H_impl(mesh, mv, d_X, d_Y, prec, stream, false);
  return MFB_OK;
  MFB_CATCH
}

int mfb_mv_zero(const mfb_mv* mv, double* d_Y, void* stream) {
  MFB_TRY
  if (!mv || !d_Y) fail(MFB_EINVAL, "null argument");
  const int rc = mfb::gpu::launch_zero(d_Y, mv->plan.block_offset.back(), stream);
  if (rc != 0) fail(MFB_EHIP, std::string("kernel launch: ") + hipGetErrorString((hipError_t)rc));
  return MFB_OK;
  MFB_CATCH
}

int mfb_apply_H_tuned(const mfb_mesh* mesh, const mfb_mv* mv, const double* d_X, double* d_Y,
                      const mfb_tune* tune, void* d_work, void* stream) {
  MFB_TRY
  check_apply_args(mesh, mv, d_X, d_Y);
  if (!tune) fail(MFB_EINVAL, "null tune");
  if (tune->prec < 0 || tune->prec > 3) fail(MFB_EINVAL, "unknown precision");
  if (tune->kernel < 0 || tune->kernel > 9) fail(MFB_EINVAL, "kernel must be in 0..9");
  if (tune->grid < 0) fail(MFB_EINVAL, "negative grid");
  if ((tune->kernel == 0 || tune->kernel == 2) &&
      (tune->grid > 64 || (tune->grid & (tune->grid - 1)) != 0))
    fail(MFB_EINVAL, "kernels 0 and 2 take grid = 0 or a power of two up to 64");
  if (mesh->plan.curved && tune->kernel != 0 && tune->kernel != 2 && tune->kernel != 7)
    fail(MFB_EUNSUPPORTED, "curved cells run the fused kernels only (0, 2 and 7)");
  if (tune->kernel == 8 && !mfb::gpu::reg_kernel_supported(mesh->plan.p, tune->prec, mesh->plan.curved))
    fail(MFB_EUNSUPPORTED, "kernel 8 takes p <= 2, box cells and the vector-ALU precisions");
  if (tune->kernel == 9 && (mesh->plan.p < 2 || (tune->prec != MFB_FP64 && tune->prec != MFB_FP32)))
    fail(MFB_EUNSUPPORTED, "kernel 9 takes p >= 2 and the vector-ALU precisions");
  if ((tune->kernel & 1) && tune->kernel != 7 && tune->kernel != 9 && !d_work)
    fail(MFB_EINVAL, "the queue kernels need the workspace");
  mfb::gpu::ApplyParams a;
  fill_apply_params(mesh, mv, d_X, d_Y, a);
  a.counters = (int32_t*)d_work;
  a.grid = tune->grid;
  const int rc =
      mfb::gpu::launch_apply(a, mesh->plan.p, tune->prec, tune->kernel, mv->plan.block_offset.back(), stream);
  if (rc == -2) fail(MFB_EUNSUPPORTED, "precision not implemented by the library");
  if (rc != 0) fail(MFB_EHIP, std::string("kernel launch: ") + hipGetErrorString((hipError_t)rc));
  return MFB_OK;
  MFB_CATCH
}

int mfb_create_closure(const mfb_mv* x, mfb_mv** out) {
  MFB_TRY
  if (!x || !out) fail(MFB_EINVAL, "null argument");
  *out = nullptr;
  if (x->source) fail(MFB_EINVAL, "the closure of a closure layout is not supported");
  auto* v = new mfb_mv();
  try {
    mfb::plan_closure(v->plan, x->plan, x->mesh->plan);
    v->mesh = x->mesh;
    v->source = x;
    v->lay = mv_layout(v->plan);
    v->work_bytes = kCounterBytes + sizeof(double) * (size_t)(v->plan.part_doubles + v->plan.ndiag);
    v->pattern_id = g_next_pattern_id++;
  } catch (...) {
    delete v;
    throw;
  }
  *out = v;
  return MFB_OK;
  MFB_CATCH
}

int mfb_apply_op(const mfb_mesh* mesh, const mfb_mv* x, const mfb_mv* y, int op, const double* d_X,
                 double* d_Y, int prec, void* stream) {
  MFB_TRY
  check_apply_args(mesh, x, d_X, d_Y);
  if (!y) fail(MFB_EINVAL, "null argument");
  const bool closure_dest = y->source && same_pattern(y->source, x);
  if (!same_pattern(y, x) && !closure_dest)
    fail(MFB_EPATTERN, "y must have the pattern of x or be its closure");
  if (!y->bound) fail(MFB_ESTATE, "destination layout metadata not bound");
  if (op != MFB_OP_H && op != MFB_OP_M) fail(MFB_EINVAL, "unknown operator");
  if (prec < 0 || prec > 3) fail(MFB_EINVAL, "unknown precision");
  mfb::gpu::ApplyParams a;
  fill_apply_params(mesh, x, d_X, d_Y, a);
  if (closure_dest) a.rowoff_out = (const int32_t*)((const char*)y->d_meta + y->lay.off_dest_rowoff);
  const int rc = mfb::gpu::launch_apply_op(a, mesh->plan.p, prec, op, y->plan.block_offset.back(),
                                           stream);
  if (rc == -2) fail(MFB_EUNSUPPORTED, "precision not implemented by the library");
  if (rc != 0) fail(MFB_EHIP, std::string("kernel launch: ") + hipGetErrorString((hipError_t)rc));
  return MFB_OK;
  MFB_CATCH
}

int mfb_energy(int32_t M, const double* d_Mbar, const double* d_Hbar, double* d_E, void* d_work,
               void* stream) {
  MFB_TRY
  if (!d_Mbar || !d_Hbar || !d_E || !d_work) fail(MFB_EINVAL, "null argument");
  if (M <= 0) fail(MFB_EINVAL, "M must be positive");
  if (((uintptr_t)d_work & 7) != 0) fail(MFB_EINVAL, "d_work must be 8-byte aligned");
  const int rc = mfb::gpu::launch_energy(M, d_Mbar, d_Hbar, d_E, (double*)d_work, stream);
  if (rc != 0) fail(MFB_EHIP, std::string("kernel launch: ") + hipGetErrorString((hipError_t)rc));
  return MFB_OK;
  MFB_CATCH
}

// Two layouts with the same rows and columns: the same pattern, one the
// closure of the other, or two closures of the same pattern.
static bool same_rows_and_columns(const mfb_mv* a, const mfb_mv* b) {
  if (same_pattern(a, b)) return true;
  if (a->source && same_pattern(a->source, b)) return true;
  if (b->source && same_pattern(b->source, a)) return true;
  return a->source && b->source && same_pattern(a->source, b->source);
}

static mfb::gpu::BlockView block_view(const mfb_mv* v) {
  const char* mb = (const char*)v->d_meta;
  mfb::gpu::BlockView b;
  b.rowptr = (const int64_t*)(mb + v->lay.off_rowptr);
  b.blk_off = (const int64_t*)(mb + v->lay.off_blk_off);
  b.blk_col0 = (const int32_t*)(mb + v->lay.off_blk_col0);
  b.blk_w = (const int32_t*)(mb + v->lay.off_blk_w);
  b.blk_row = (const int32_t*)(mb + v->lay.off_blk_row);
  b.nblocks = (int64_t)v->plan.colidx.size();
  return b;
}

int mfb_mmult(const mfb_mv* a, const mfb_mv* c, const double* d_A, const double* d_B, double alpha,
              double beta, double* d_C, int accumulate, void* stream) {
  MFB_TRY
  if (!a || !c || !d_A || !d_B || !d_C) fail(MFB_EINVAL, "null argument");
  if (!same_rows_and_columns(a, c)) fail(MFB_EPATTERN, "a and c must share rows and columns");
  if (!a->bound || !c->bound) fail(MFB_ESTATE, "layout metadata not bound");
  if (d_A == d_C) fail(MFB_EINVAL, "A and C must not alias");
  if (!std::isfinite(alpha) || !std::isfinite(beta)) fail(MFB_EINVAL, "alpha and beta must be finite");
  mfb::gpu::MmultParams q;
  q.A = d_A;
  q.B = d_B;
  q.C = d_C;
  q.a = block_view(a);
  q.c = block_view(c);
  q.M = a->plan.M;
  q.alpha = alpha;
  q.beta = beta;
  q.accumulate = accumulate ? 1 : 0;
  q.max_rows = 0;
  const auto& rb = c->mesh->plan.rb_start;
  for (size_t r = 0; r + 1 < rb.size(); ++r) q.max_rows = std::max<int64_t>(q.max_rows, rb[r + 1] - rb[r]);
  const int rc = mfb::gpu::launch_mmult(q, stream);
  if (rc != 0) fail(MFB_EHIP, std::string("kernel launch: ") + hipGetErrorString((hipError_t)rc));
  return MFB_OK;
  MFB_CATCH
}

int mfb_mv_axpy(const mfb_mv* mv, double alpha, const double* d_X, double* d_Y, void* stream) {
  MFB_TRY
  if (!mv || !d_X || !d_Y) fail(MFB_EINVAL, "null argument");
  if (!std::isfinite(alpha)) fail(MFB_EINVAL, "alpha must be finite");
  const int rc = mfb::gpu::launch_axpy(mv->plan.block_offset.back(), alpha, d_X, d_Y, stream);
  if (rc != 0) fail(MFB_EHIP, std::string("kernel launch: ") + hipGetErrorString((hipError_t)rc));
  return MFB_OK;
  MFB_CATCH
}

int mfb_mv_scale_columns(const mfb_mv* mv, const double* d_scale, double* d_X, void* stream) {
  MFB_TRY
  if (!mv || !d_scale || !d_X) fail(MFB_EINVAL, "null argument");
  if (!mv->bound) fail(MFB_ESTATE, "layout metadata not bound");
  const int rc = mfb::gpu::launch_scale_columns(block_view(mv), d_scale, d_X, stream);
  if (rc != 0) fail(MFB_EHIP, std::string("kernel launch: ") + hipGetErrorString((hipError_t)rc));
  return MFB_OK;
  MFB_CATCH
}

int mfb_mv_dot(const mfb_mv* mv, const double* d_X, const double* d_Y, double* d_out, void* d_work,
               void* stream) {
  MFB_TRY
  if (!mv || !d_X || !d_Y || !d_out || !d_work) fail(MFB_EINVAL, "null argument");
  if (((uintptr_t)d_work & 7) != 0) fail(MFB_EINVAL, "d_work must be 8-byte aligned");
  const int rc = mfb::gpu::launch_dot(mv->plan.block_offset.back(), d_X, d_Y, d_out,
                                      (double*)d_work, stream);
  if (rc != 0) fail(MFB_EHIP, std::string("kernel launch: ") + hipGetErrorString((hipError_t)rc));
  return MFB_OK;
  MFB_CATCH
}

static void tmmult_enqueue(const mfb_mv* mv, const double* d_X, const double* d_Y, double* d_S,
                           double* d_trace, void* d_work, void* stream, int unit_steps = 0,
                           int long_steps = 0) {
  const auto& p = mv->plan;
  const char* mb = (const char*)mv->d_meta;
  mfb::gpu::TmParams t;
  t.X = d_X;
  t.Y = d_Y;
  t.units = (const mfb::TmUnit*)(mb + mv->lay.off_units);
  t.nunits = (int64_t)p.units.size();
  for (int c = 0; c < 4; ++c) t.class_end[c] = p.tm_class_end[c];
  t.tasks = (const mfb::TmTask*)(mb + mv->lay.off_tasks);
  t.task_blk = (const mfb::TaskBlk*)(mb + mv->lay.off_task_blk);
  t.task_part = (const int64_t*)(mb + mv->lay.off_task_part);
  for (int c = 0; c < 3; ++c) t.task_class_end[c] = p.task_class_end[c];
  t.part = (double*)((char*)d_work + kCounterBytes);
  t.tdiag = t.part + p.part_doubles;
  t.ndiag = p.ndiag;
  t.fold_trace = p.tasks.empty() ? 1 : 0;
  t.pair_tab = (const int32_t*)(mb + mv->lay.off_pair_tab);
  t.pair_ptr = (const int32_t*)(mb + mv->lay.off_pair_ptr);
  t.pair_list = (const int64_t*)(mb + mv->lay.off_pair_list);
  t.cb_of_col = (const int32_t*)(mb + mv->lay.off_cb_of_col);
  t.cb_start = (const int32_t*)(mb + mv->lay.off_cb_start);
  t.s2 = (const mfb::S2Desc*)(mb + mv->lay.off_s2);
  t.max_pair_parts = 0;
  for (size_t i = 0; i + 1 < p.pair_ptr.size(); ++i)
    t.max_pair_parts = std::max<int64_t>(t.max_pair_parts, p.pair_ptr[i + 1] - p.pair_ptr[i]);
  t.M = p.M;
  t.ncb = p.ncb;

  t.S = d_S;
  t.trace = d_trace;
  const int rc = mfb::gpu::launch_tmmult(t, stream, unit_steps, long_steps);
  if (rc != 0) fail(MFB_EHIP, std::string("kernel launch: ") + hipGetErrorString((hipError_t)rc));
}

int mfb_tmmult(const mfb_mv* mv, const double* d_X, const double* d_Y, double* d_S, double* d_trace,
               void* d_work, void* stream) {
  MFB_TRY
  if (!mv || !d_X || !d_Y || !d_S || !d_trace || !d_work) fail(MFB_EINVAL, "null argument");
  if (!mv->bound) fail(MFB_ESTATE, "layout metadata not bound");
  if (((uintptr_t)d_work & 255) != 0) fail(MFB_EINVAL, "d_work must be 256-byte aligned");
  tmmult_enqueue(mv, d_X, d_Y, d_S, d_trace, d_work, stream);
  return MFB_OK;
  MFB_CATCH
}

int mfb_tmmult_tuned(const mfb_mv* mv, const double* d_X, const double* d_Y, double* d_S,
                     double* d_trace, void* d_work, const mfb_tm_tune* tune, void* stream) {
  MFB_TRY
  if (!mv || !d_X || !d_Y || !d_S || !d_trace || !d_work || !tune) fail(MFB_EINVAL, "null argument");
  auto steps_ok = [](int32_t s) { return s == 0 || s == 4 || s == 8 || s == 16; };
  if (!steps_ok(tune->unit_steps) || !steps_ok(tune->long_steps))
    fail(MFB_EINVAL, "row steps must be 0, 4, 8 or 16");
  if (!mv->bound) fail(MFB_ESTATE, "layout metadata not bound");
  if (((uintptr_t)d_work & 255) != 0) fail(MFB_EINVAL, "d_work must be 256-byte aligned");
  tmmult_enqueue(mv, d_X, d_Y, d_S, d_trace, d_work, stream, tune->unit_steps, tune->long_steps);
  return MFB_OK;
  MFB_CATCH
}

int mfb_tmmult_noalloc(const mfb_mv* mv, const double* d_X, const double* d_Y, double* d_S,
                       double* d_trace, void* stream) {
  MFB_TRY
  if (!mv || !d_X || !d_Y || !d_S || !d_trace) fail(MFB_EINVAL, "null argument");
  if (mv->work_bytes > mfb::gpu::kScratchBytes)
    fail(MFB_EINVAL, "the overlap workspace of this layout (" + std::to_string(mv->work_bytes) +
                         " bytes) exceeds the fixed scratch of " +
                         std::to_string(mfb::gpu::kScratchBytes) +
                         " bytes; use mfb_tmmult with a workspace");
  if (!mv->bound) fail(MFB_ESTATE, "layout metadata not bound");
  void* w = nullptr;
  const int rc = mfb::gpu::scratch_address(&w);
  if (rc != 0) fail(MFB_EHIP, std::string("scratch address: ") + hipGetErrorString((hipError_t)rc));
  tmmult_enqueue(mv, d_X, d_Y, d_S, d_trace, w, stream);
  return MFB_OK;
  MFB_CATCH
}

int mfb_mv_update(const mfb_mv* mv, double* d_X, const double* d_Y, const double* d_S,
                  const double* d_S2, double tau, void* stream) {
  MFB_TRY
  if (!mv || !d_X || !d_Y || !d_S || !d_S2) fail(MFB_EINVAL, "null argument");
  if (mv->source) fail(MFB_EINVAL, "the update works on X's own layout, not a closure");
  if (!mv->bound) fail(MFB_ESTATE, "layout metadata not bound");
  if (!std::isfinite(tau)) fail(MFB_EINVAL, "tau must be finite");
  const char* mb = (const char*)mv->d_meta;
  mfb::gpu::UpdateParams u;
  u.X = d_X;
  u.Y = d_Y;
  u.S = d_S;
  u.S2 = d_S2;
  u.blk_off = (const int64_t*)(mb + mv->lay.off_blk_off);
  u.blk_col0 = (const int32_t*)(mb + mv->lay.off_blk_col0);
  u.blk_w = (const int32_t*)(mb + mv->lay.off_blk_w);
  u.nblocks = (int64_t)mv->plan.colidx.size();
  u.M = mv->plan.M;
  u.tau = tau;
  const int rc = mfb::gpu::launch_update(u, stream);
  if (rc != 0) fail(MFB_EHIP, std::string("kernel launch: ") + hipGetErrorString((hipError_t)rc));
  return MFB_OK;
  MFB_CATCH
}

int mfb_probe_fp64_fma(double* d_out, int64_t blocks, int32_t iters, void* stream) {
  MFB_TRY
  if (!d_out) fail(MFB_EINVAL, "null output");
  if (blocks < 1 || blocks > (int64_t(1) << 31) - 1 || iters < 1) fail(MFB_EINVAL, "blocks and iters must be positive");
  const int rc = mfb::gpu::launch_probe_fma(d_out, blocks, iters, stream);
  if (rc != 0) fail(MFB_EHIP, std::string("kernel launch: ") + hipGetErrorString((hipError_t)rc));
  return MFB_OK;
  MFB_CATCH
}

}  // extern "C"
