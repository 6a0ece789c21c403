// C ABI of hipbc: argument checking, object lifetime, error reporting.
// Every entry point catches all C++ exceptions and turns them into codes.
#include <algorithm>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>

#include "device.hpp"
#include "hbc_internal.hpp"

struct hbc_grid {
  hbc::Grid g;
};
struct hbc_program {
  hbc::Program p;
};
struct hbc_plan {
  hbc::Plan p;
  std::mutex csc_mu;
  bool csc_ready = false;
};
struct hbc_graph {
  void* g = nullptr;
};
struct hbc_consumer {
  const hbc_plan* plan = nullptr;
  hbc::ConsumerHost host;
  void* dev = nullptr;
};
struct hbc_batch {
  hbc::Batch* b = nullptr;
  std::vector<const hbc::Plan*> plans;
};

namespace hbc {

namespace {
thread_local std::string g_last_error;

struct Fail {
  int code;
  std::string msg;
};
}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }
[[noreturn]] void fail(int code, const std::string& msg) { throw Fail{code, msg}; }

template <class F>
int guard(F&& f) {
  try {
    g_last_error.clear();
    f();
    return HBC_OK;
  } catch (const Fail& e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "out of host memory";
    return HBC_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return HBC_EINVAL;
  } catch (...) {
    g_last_error = "unknown error";
    return HBC_EINVAL;
  }
}

static void need(bool ok, const char* what) {
  if (!ok) fail(HBC_EINVAL, what);
}

// ---- positions -> lattice indices (stepped slices, Sec. IV-A-1) ----------------
static int64_t floor_div(int64_t a, int64_t b) { return a / b - ((a % b != 0) && ((a < 0) != (b < 0))); }
static int64_t ceil_div(int64_t a, int64_t b) { return -floor_div(-a, b); }
static int64_t floor_mod(int64_t a, int64_t b) { return a - floor_div(a, b) * b; }

// Index of the first lattice point >= p along dimension d.
static int64_t index_at_or_after(const Grid& g, int d, int64_t p) { return ceil_div(p - g.res[d], g.step[d]); }

// Index of lattice point p (HBC_ERANGE if p is not one).
static int64_t index_of(const Grid& g, int d, int64_t p) {
  if (floor_mod(p - g.res[d], g.step[d]) != 0)
    fail(HBC_ERANGE, "position " + std::to_string(p) + " is not a point of the grid's lattice along dimension " +
                         std::to_string(d));
  return (p - g.res[d]) / g.step[d];
}

// A box of positions -> the box of lattice indices of the points it holds.
static Box to_box(const Grid& g, const hbc_box* b) {
  need(b != nullptr, "rows box is NULL");
  Box r;
  r.nd = g.nd;
  for (int d = 0; d < g.nd; ++d) {
    need(b->hi[d] >= b->lo[d], "box with hi < lo");
    r.lo[d] = index_at_or_after(g, d, b->lo[d]);
    r.hi[d] = std::max(r.lo[d], index_at_or_after(g, d, b->hi[d]));
  }
  return r;
}

// A column given as a row-major linear index over the global box of
// positions -> the linear index over the global box of lattice indices
// (-1, padding, stays -1).
static int64_t to_col(const Grid& g, int64_t lin) {
  if (lin < 0 || g.identity_lattice()) return lin;
  int64_t c[HBC_MAX_DIM];
  for (int d = g.nd - 1; d >= 0; --d) {
    const int64_t n = g.phi[d] - g.plo[d];
    c[d] = g.plo[d] + lin % n;
    lin /= n;
  }
  if (lin != 0) fail(HBC_ERANGE, "column index outside the global box");
  int64_t out = 0;
  for (int d = 0; d < g.nd; ++d) out = out * (g.hi[d] - g.lo[d]) + (index_of(g, d, c[d]) - g.lo[d]);
  return out;
}

static void to_cols(const Grid& g, std::vector<int64_t>& cols) {
  if (g.identity_lattice()) return;
  for (int64_t& c : cols) c = to_col(g, c);
}

static void finish_grid(Grid& g) {
  int64_t n = 0;
  for (Block& b : g.blocks) {
    b.first_cell = n;
    int64_t s = 1;
    for (int d = g.nd - 1; d >= 0; --d) {
      b.stride[d] = s;
      s *= b.full.extent(d);
    }
    b.cells = s;
    n += s;
  }
  g.ncells = n;
}

static int add_sub(hbc_program* p, Sub&& s, int32_t* sub_id) {
  p->p.subs.push_back(std::move(s));
  if (sub_id) *sub_id = (int32_t)p->p.subs.size() - 1;
  return HBC_OK;
}

}  // namespace hbc

using namespace hbc;

extern "C" {

const char* hbc_last_error(void) { return g_last_error.c_str(); }

// ---- grid -----------------------------------------------------------------------------
int hbc_grid_create(int32_t ndim, const int64_t* lo, const int64_t* hi, hbc_grid** out) {
  return guard([&] {
    need(out && lo && hi, "NULL argument");
    need(ndim >= 1 && ndim <= HBC_MAX_DIM, "ndim must be in [1, 6]");
    for (int d = 0; d < ndim; ++d) need(hi[d] > lo[d], "global box must be non-empty");
    auto g = std::make_unique<hbc_grid>();
    g->g.nd = ndim;
    for (int d = 0; d < ndim; ++d) {
      g->g.lo[d] = g->g.plo[d] = lo[d];
      g->g.hi[d] = g->g.phi[d] = hi[d];
    }
    *out = g.release();
  });
}

int hbc_grid_add_block(hbc_grid* gh, const hbc_slice* full, const hbc_slice* data, int32_t* block_id) {
  return guard([&] {
    need(gh && full && data, "NULL argument");
    Grid& live = gh->g;
    for (int d = 0; d < live.nd; ++d) need(full[d].step >= 1 && data[d].step >= 1, "slice steps must be >= 1");
    // work on a copy: the grid (and, for its first block, its lattice) changes
    // only if the block is accepted
    Grid g = live;
    if (!g.lattice_set) {  // the first block fixes the grid's lattice
      for (int d = 0; d < g.nd; ++d) {
        g.step[d] = full[d].step;
        g.res[d] = floor_mod(full[d].start, full[d].step);
        g.lo[d] = index_at_or_after(g, d, g.plo[d]);
        g.hi[d] = index_at_or_after(g, d, g.phi[d]);
      }
      g.lattice_set = true;
    }
    Block b;
    b.full.nd = b.data.nd = g.nd;
    for (int d = 0; d < g.nd; ++d) {
      if (full[d].step != g.step[d] || data[d].step != g.step[d] || floor_mod(full[d].start, g.step[d]) != g.res[d] ||
          floor_mod(data[d].start, g.step[d]) != g.res[d])
        fail(HBC_EUNSUPPORTED,
             "the full and data slices of every block of a grid must lie on one lattice (same step, starts "
             "congruent modulo the step); other step patterns are not implemented");
      need(g.plo[d] <= full[d].start && full[d].start <= data[d].start && data[d].start < data[d].stop &&
               data[d].stop <= full[d].stop && full[d].stop <= g.phi[d],
           "need lo <= full.start <= data.start < data.stop <= full.stop <= hi");
      b.full.lo[d] = index_of(g, d, full[d].start);
      b.full.hi[d] = index_at_or_after(g, d, full[d].stop);
      b.data.lo[d] = index_of(g, d, data[d].start);
      b.data.hi[d] = index_at_or_after(g, d, data[d].stop);
    }
    for (const Block& o : g.blocks) need(!intersects(o.full, b.full), "block full regions overlap");
    g.blocks.push_back(b);
    finish_grid(g);
    need(g.ncells < (int64_t(1) << 40), "grid too large");
    live = std::move(g);
    if (block_id) *block_id = (int32_t)live.blocks.size() - 1;
  });
}

int64_t hbc_grid_cells(const hbc_grid* g) { return g ? g->g.ncells : 0; }

int hbc_grid_block_cells(const hbc_grid* g, int32_t b, int64_t* first, int64_t* n) {
  return guard([&] {
    need(g && first && n, "NULL argument");
    need(b >= 0 && b < (int32_t)g->g.blocks.size(), "block out of range");
    *first = g->g.blocks[b].first_cell;
    *n = g->g.blocks[b].cells;
  });
}

void hbc_grid_destroy(hbc_grid* g) { delete g; }

int hbc_cs_grid_create(int64_t N, int64_t h, hbc_grid** out) {
  return guard([&] {
    need(out != nullptr, "NULL argument");
    need(N >= 4 && h >= 1 && 2 * h <= N,
         "cubed sphere needs N >= 4 and 1 <= h <= N/2 (deeper ghost layers leave the face's gnomonic chart)");
    auto g = std::make_unique<hbc_grid>();  // freed if a later allocation throws
    Grid& G = g->g;
    G.nd = 3;
    G.lo[0] = 0; G.hi[0] = 6;
    G.lo[1] = G.lo[2] = -h;
    G.hi[1] = G.hi[2] = N + h;
    for (int f = 0; f < 6; ++f) {
      Block b;
      b.full.nd = b.data.nd = 3;
      b.full.lo[0] = b.data.lo[0] = f;
      b.full.hi[0] = b.data.hi[0] = f + 1;
      for (int d = 1; d < 3; ++d) {
        b.full.lo[d] = -h; b.full.hi[d] = N + h;
        b.data.lo[d] = 0; b.data.hi[d] = N;
      }
      G.blocks.push_back(b);
    }
    finish_grid(G);
    *out = g.release();
  });
}

int hbc_cart_grid_create(const int32_t* nb, const int64_t* n, int64_t h, hbc_grid** out) {
  return guard([&] {
    need(out && nb && n, "NULL argument");
    need(h >= 1, "halo must be >= 1");
    for (int d = 0; d < 3; ++d) need(nb[d] >= 1 && n[d] >= 1, "block counts and sizes must be >= 1");
    auto g = std::make_unique<hbc_grid>();  // freed if a later allocation throws
    Grid& G = g->g;
    G.nd = 4;
    const int64_t nblk = (int64_t)nb[0] * nb[1] * nb[2];
    G.lo[0] = 0; G.hi[0] = nblk;
    for (int d = 0; d < 3; ++d) {
      G.lo[d + 1] = -h;
      G.hi[d + 1] = n[d] + h;
    }
    for (int64_t b = 0; b < nblk; ++b) {
      Block B;
      B.full.nd = B.data.nd = 4;
      B.full.lo[0] = B.data.lo[0] = b;
      B.full.hi[0] = B.data.hi[0] = b + 1;
      for (int d = 0; d < 3; ++d) {
        B.full.lo[d + 1] = -h; B.full.hi[d + 1] = n[d] + h;
        B.data.lo[d + 1] = 0; B.data.hi[d + 1] = n[d];
      }
      G.blocks.push_back(B);
    }
    finish_grid(G);
    *out = g.release();
  });
}

// ---- program --------------------------------------------------------------------------
int hbc_program_create(const hbc_grid* g, hbc_program** out) {
  return guard([&] {
    need(g && out, "NULL argument");
    need(!g->g.blocks.empty(), "grid has no blocks");
    auto p = std::make_unique<hbc_program>();
    p->p.grid = g->g;
    *out = p.release();
  });
}

void hbc_program_destroy(hbc_program* p) { delete p; }

int hbc_program_set_flags(hbc_program* p, uint32_t flags) {
  return guard([&] {
    need(p != nullptr, "NULL argument");
    need((flags & ~(HBC_STRICT_COVER | HBC_ALLOW_OVERLAP_SUM)) == 0, "unknown program flag");
    p->p.flags = flags;
  });
}

int hbc_program_set_consumer(hbc_program* p, int32_t noffsets, const int64_t* offsets) {
  return guard([&] {
    need(p != nullptr, "NULL argument");
    need(noffsets >= 0, "noffsets must be >= 0");
    need(noffsets == 0 || offsets != nullptr, "NULL offsets");
    const Grid& g = p->p.grid;
    p->p.consumer.assign(offsets, offsets + (size_t)noffsets * g.nd);
    for (size_t k = 0; k < p->p.consumer.size(); ++k) {  // positions -> lattice steps
      const int d = (int)(k % (size_t)g.nd);
      need(p->p.consumer[k] % g.step[d] == 0, "consumer offsets must be multiples of the grid's step");
      p->p.consumer[k] /= g.step[d];
    }
  });
}

int hbc_program_add_map(hbc_program* p, const hbc_box* rows, const int64_t* M, const int64_t* offset, double weight,
                        const int32_t* rot, int32_t* sub_id) {
  return guard([&] {
    need(p && M && offset, "NULL argument");
    Sub s;
    s.kind = SUB_MAP;
    const Grid& g = p->p.grid;
    s.rows = to_box(g, rows);
    const int nd = g.nd;
    // col = M row + offset in positions; with row = res + step k (component-
    // wise) the map in lattice indices has M'[i][j] = M[i][j] step[j] / step[i]
    // and offset'[i] = (sum_j M[i][j] res[j] + offset[i] - res[i]) / step[i],
    // both required to be integers
    for (int i = 0; i < nd; ++i) {
      int64_t o = offset[i] - g.res[i];
      for (int j = 0; j < nd; ++j) {
        const int64_t m = M[i * nd + j] * g.step[j];
        need(m % g.step[i] == 0, "map does not send lattice points to lattice points");
        s.M[i * nd + j] = m / g.step[i];
        o += M[i * nd + j] * g.res[j];
      }
      need(floor_mod(o, g.step[i]) == 0, "map does not send lattice points to lattice points");
      s.off[i] = floor_div(o, g.step[i]);
    }
    s.w = weight;
    s.rot = rot_code(rot);
    need(s.rot >= 0, "rot must be a 2x2 signed permutation");
    add_sub(p, std::move(s), sub_id);
  });
}

int hbc_program_box_rows(const hbc_program* p, const hbc_box* rows, int64_t* n) {
  return guard([&] {
    need(p && n, "NULL argument");
    *n = to_box(p->p.grid, rows).count();
  });
}

int hbc_program_add_zero(hbc_program* p, const hbc_box* rows, int32_t* sub_id) {
  return guard([&] {
    need(p != nullptr, "NULL argument");
    Sub s;
    s.kind = SUB_ZERO;
    s.rows = to_box(p->p.grid, rows);
    add_sub(p, std::move(s), sub_id);
  });
}

int hbc_program_add_zero_rest(hbc_program* p, int32_t block, int32_t* sub_id) {
  return guard([&] {
    need(p != nullptr, "NULL argument");
    need(block >= 0 && block < (int32_t)p->p.grid.blocks.size(), "block out of range");
    Sub s;
    s.kind = SUB_ZERO_REST;
    s.block = block;
    s.rows.nd = p->p.grid.nd;
    add_sub(p, std::move(s), sub_id);
  });
}

int hbc_program_add_ell(hbc_program* p, const hbc_box* rows, int32_t width, const int64_t* cols, const double* vals,
                        const int32_t* rot, int32_t* sub_id) {
  return guard([&] {
    need(p != nullptr, "NULL argument");
    need(width >= 1 && width <= 64, "ELL width must be in [1, 64]");
    Sub s;
    s.kind = SUB_ELL;
    s.rows = to_box(p->p.grid, rows);
    const int64_t n = s.rows.count() * width;
    need(n == 0 || (cols && vals), "NULL cols / vals");
    s.width = width;
    s.cols.assign(cols, cols + n);
    to_cols(p->p.grid, s.cols);
    s.vals.assign(vals, vals + n);
    s.rot = rot_code(rot);
    need(s.rot >= 0, "rot must be a 2x2 signed permutation");
    add_sub(p, std::move(s), sub_id);
  });
}

int hbc_program_add_csr(hbc_program* p, const hbc_box* rows, const int64_t* row_ptr, const int64_t* cols,
                        const double* vals, const int32_t* rot, int32_t* sub_id) {
  return guard([&] {
    need(p && row_ptr, "NULL argument");
    Sub s;
    s.kind = SUB_CSR;
    s.rows = to_box(p->p.grid, rows);
    const int64_t nr = s.rows.count();
    need(row_ptr[0] == 0, "row_ptr[0] must be 0");
    for (int64_t k = 0; k < nr; ++k) need(row_ptr[k + 1] >= row_ptr[k], "row_ptr must be non-decreasing");
    const int64_t nnz = row_ptr[nr];
    need(nnz == 0 || (cols && vals), "NULL cols / vals");
    s.ptr.assign(row_ptr, row_ptr + nr + 1);
    s.cols.assign(cols, cols + nnz);
    to_cols(p->p.grid, s.cols);
    s.vals.assign(vals, vals + nnz);
    s.rot = rot_code(rot);
    need(s.rot >= 0, "rot must be a 2x2 signed permutation");
    add_sub(p, std::move(s), sub_id);
  });
}

int hbc_program_add_vector(hbc_program* p, const hbc_box* rows, int64_t ninner, const double* values,
                           int32_t* sub_id) {
  return guard([&] {
    need(p != nullptr, "NULL argument");
    need(ninner >= 1, "ninner must be >= 1");
    Sub s;
    s.kind = SUB_VEC;
    s.rows = to_box(p->p.grid, rows);
    const int64_t n = s.rows.count() * ninner;
    need(n == 0 || values, "NULL values");
    s.ninner = ninner;
    s.b.assign(values, values + n);
    add_sub(p, std::move(s), sub_id);
  });
}

int hbc_program_add_data_csr(hbc_program* p, const hbc_box* rows, const int64_t* row_ptr, const int64_t* cols,
                             const double* vals, int32_t* sub_id) {
  return guard([&] {
    need(p && row_ptr, "NULL argument");
    DataSub s;
    s.rows = to_box(p->p.grid, rows);
    const int64_t nr = s.rows.count();
    need(row_ptr[0] == 0, "row_ptr[0] must be 0");
    for (int64_t k = 0; k < nr; ++k) need(row_ptr[k + 1] >= row_ptr[k], "row_ptr must be non-decreasing");
    const int64_t nnz = row_ptr[nr];
    need(nnz == 0 || (cols && vals), "NULL cols / vals");
    s.ptr.assign(row_ptr, row_ptr + nr + 1);
    s.cols.assign(cols, cols + nnz);
    to_cols(p->p.grid, s.cols);
    s.vals.assign(vals, vals + nnz);
    p->p.dsubs.push_back(std::move(s));
    if (sub_id) *sub_id = (int32_t)(p->p.dsubs.size() - 1);
  });
}

int hbc_cs_program_add_quadrature(hbc_program* p, int64_t N, int64_t h, int32_t q, int32_t vector) {
  return guard([&] {
    need(p != nullptr, "NULL argument");
    cs_add_quadrature(p->p, N, h, q, vector);
  });
}

int hbc_cs_program_add_edge_average(hbc_program* p, int64_t Np) {
  return guard([&] {
    need(p != nullptr, "NULL argument");
    cs_add_edge_average(p->p, Np);
  });
}

int hbc_cs_program_add(hbc_program* p, int64_t N, int64_t h, int32_t mode, int32_t vector, const int32_t* base,
                       const double* w) {
  return guard([&] {
    need(p != nullptr, "NULL argument");
    cs_add_program(p->p, N, h, mode, vector, base, w);
  });
}

int hbc_cart_program_add_halo(hbc_program* p, const int32_t* nb, const int64_t* n, int64_t h, int32_t periodic) {
  return guard([&] {
    need(p && nb && n, "NULL argument");
    cart_add_halo(p->p, nb, n, h, periodic);
  });
}

// ---- plan -----------------------------------------------------------------------------
int hbc_plan_create(const hbc_program* prog, const hbc_layout* layout, int32_t dtype, uint32_t flags,
                    hbc_plan** out) {
  hbc_plan* pl = nullptr;
  int rc = guard([&] {
    need(prog && layout && out, "NULL argument");
    need(dtype == HBC_F64 || dtype == HBC_F32, "dtype must be HBC_F64 or HBC_F32");
    need((flags & ~(HBC_PLAN_HOST_ONLY | HBC_PLAN_NO_WINDOWS)) == 0, "unknown plan flag");
    pl = new hbc_plan;
    Layout lay;
    lay.inner = layout->inner;
    lay.order = layout->order;
    lay.vec_len = layout->vec_len;
    lay.vec_lo = layout->vec_lo;
    lay.vec_stride = layout->vec_stride;
    pl->p.flags = flags;
    compile_plan(prog->p, lay, dtype, pl->p);
    if (!(flags & HBC_PLAN_HOST_ONLY)) device_upload_plan(pl->p);
    *out = pl;
    pl = nullptr;
  });
  if (pl) {
    device_free_plan(pl->p);
    delete pl;
  }
  return rc;
}

void hbc_plan_destroy(hbc_plan* plan) {
  if (!plan) return;
  device_free_plan(plan->p);
  delete plan;
}

int hbc_plan_stats(const hbc_plan* plan, hbc_stats* out) {
  return guard([&] {
    need(plan && out, "NULL argument");
    *out = plan->p.stats;
    out->table_bytes = (int64_t)plan->p.dev_bytes;
  });
}

int hbc_plan_row(const hbc_plan* plan, int64_t ghost_cell, int64_t l, int32_t cap, int64_t* cols, double* vals,
                 int32_t* nnz, double* b, int32_t* kind, int32_t* rot) {
  return guard([&] {
    need(plan && nnz && b && kind && rot, "NULL argument");
    need(cap == 0 || (cols && vals), "NULL cols / vals");
    need(ghost_cell >= 0 && ghost_cell < plan->p.grid.ncells, "cell out of range");
    need(l >= 0 && l < plan->p.layout.inner, "inner slot out of range");
    plan_row(plan->p, ghost_cell, l, cap, cols, vals, nnz, b, kind, rot);
  });
}

int hbc_plan_set_vector(hbc_plan* plan, int32_t sub_id, const double* values, void* stream) {
  return guard([&] {
    need(plan != nullptr, "NULL argument");
    const std::pair<int64_t, int64_t> r = plan_set_vector(plan->p, sub_id, values);
    if (!(plan->p.flags & HBC_PLAN_HOST_ONLY)) device_update_b(plan->p, r.first, r.second, stream);
  });
}

int hbc_plan_get_tune(const hbc_plan* plan, hbc_tune* out) {
  return guard([&] {
    need(plan && out, "NULL argument");
    *out = plan->p.tune;
  });
}

int hbc_plan_set_tune(hbc_plan* plan, const hbc_tune* t) {
  return guard([&] {
    need(plan && t, "NULL argument");
    build_tiles(plan->p, *t);
    if (!(plan->p.flags & HBC_PLAN_HOST_ONLY)) device_upload_tiles(plan->p);
  });
}

static void check_device_plan(const hbc_plan* plan) {
  need(plan != nullptr, "NULL plan");
  if (plan->p.flags & HBC_PLAN_HOST_ONLY) fail(HBC_EINVAL, "plan was created host-only");
}

static void check_field(const void* f) {
  need(f != nullptr, "NULL field");
  need(((uintptr_t)f & 15) == 0, "field pointer must be 16-byte aligned");
}

static void check_size(const hbc_plan* plan, int64_t nelem) {
  const int64_t want = plan->p.grid.ncells * plan->p.layout.inner;
  if (nelem != want)
    fail(HBC_EINVAL, "field has " + std::to_string(nelem) + " values, the plan needs " + std::to_string(want));
}

static void ensure_csc(hbc_plan* plan) {
  std::lock_guard<std::mutex> lk(plan->csc_mu);
  if (!plan->csc_ready) {
    build_csc(plan->p);
    device_upload_csc(plan->p);
    plan->csc_ready = true;
  }
}

int hbc_apply(const hbc_plan* plan, void* field, int64_t nelem, void* stream) {
  return guard([&] {
    check_device_plan(plan);
    check_field(field);
    check_size(plan, nelem);
    device_apply(plan->p, field, stream, false);
  });
}

int hbc_apply_adjoint(const hbc_plan* plan_c, void* grad, int64_t nelem, void* stream) {
  return guard([&] {
    check_device_plan(plan_c);
    check_field(grad);
    check_size(plan_c, nelem);
    if (plan_c->p.stats.rows_data > 0) fail(HBC_EUNSUPPORTED, "no adjoint for plans with data rows");
    auto* plan = const_cast<hbc_plan*>(plan_c);
    ensure_csc(plan);
    device_adjoint(plan->p, grad, stream);
  });
}

int hbc_apply_adjoint_noalloc(const hbc_plan* plan, void* grad, int64_t nelem, void* stream) {
  return guard([&] {
    check_device_plan(plan);
    check_field(grad);
    check_size(plan, nelem);
    if (plan->p.stats.rows_data > 0) fail(HBC_EUNSUPPORTED, "no adjoint for plans with data rows");
    {
      std::lock_guard<std::mutex> lk(const_cast<hbc_plan*>(plan)->csc_mu);
      if (!plan->csc_ready)
        fail(HBC_EINVAL, "the plan's transposed tables are not built yet: call hbc_apply_adjoint or "
                         "hbc_graph_create(HBC_OP_ADJOINT) once, where allocation is allowed");
    }
    device_adjoint_noalloc(plan->p, grad, stream);
  });
}

int hbc_plan_kernels(const hbc_plan* plan, int32_t op, char* buf, int64_t cap, int64_t* len) {
  return guard([&] {
    check_device_plan(plan);
    need(op == HBC_OP_APPLY || op == HBC_OP_ADJOINT, "op must be HBC_OP_APPLY or HBC_OP_ADJOINT");
    need(cap >= 0 && (cap == 0 || buf), "NULL buffer");
    if (op == HBC_OP_ADJOINT) {
      if (plan->p.stats.rows_data > 0) fail(HBC_EUNSUPPORTED, "no adjoint for plans with data rows");
      ensure_csc(const_cast<hbc_plan*>(plan));
    }
    std::string all;
    for (const std::string& n : device_kernel_names(plan->p, op)) all += n + "\n";
    if (len) *len = (int64_t)all.size();
    if (cap > 0) {
      const size_t n = std::min<size_t>(all.size(), (size_t)cap - 1);
      std::memcpy(buf, all.data(), n);
      buf[n] = 0;
    }
  });
}

int hbc_time_apply(const hbc_plan* plan, void* const* fields, int64_t nelem, int32_t nfields, int32_t reps,
                   void* stream, double* ms) {
  return guard([&] {
    check_device_plan(plan);
    need(fields && ms && nfields >= 1 && reps >= 1, "bad timing arguments");
    check_size(plan, nelem);
    for (int k = 0; k < nfields; ++k) check_field(fields[k]);
    *ms = device_time_apply(plan->p, fields, nfields, reps, stream);
  });
}

int hbc_plan_autotune(hbc_plan* plan, void* const* fields, int64_t nelem, int32_t nfields, const char* cache_path,
                      void* stream, double* ms) {
  return guard([&] {
    check_device_plan(plan);
    need(fields && ms && nfields >= 1, "bad tuning arguments");
    check_size(plan, nelem);
    for (int k = 0; k < nfields; ++k) check_field(fields[k]);
    *ms = device_plan_autotune(plan->p, fields, nfields, cache_path, stream);
  });
}

static void check_stencil_sizes(const hbc_plan* plan, int64_t xn, int64_t yn) {
  check_size(plan, xn);
  int64_t nd = 0;
  for (const Block& b : plan->p.grid.blocks) nd += b.data.count();
  if (yn != nd) fail(HBC_EINVAL, "y has " + std::to_string(yn) + " values, the grid has " + std::to_string(nd) + " data cells");
}

int hbc_graph_create(const hbc_plan* plan, int32_t op, void* const* fields, int64_t nelem, int32_t nfields,
                     int32_t reps, void* stream, hbc_graph** out) {
  return guard([&] {
    check_device_plan(plan);
    need(fields && out && nfields >= 1 && reps >= 1 && stream, "bad graph arguments");
    need(op == HBC_OP_APPLY || op == HBC_OP_ADJOINT, "op must be HBC_OP_APPLY or HBC_OP_ADJOINT");
    check_size(plan, nelem);
    for (int k = 0; k < nfields; ++k) check_field(fields[k]);
    if (op == HBC_OP_ADJOINT) {
      if (plan->p.stats.rows_data > 0) fail(HBC_EUNSUPPORTED, "no adjoint for plans with data rows");
      ensure_csc(const_cast<hbc_plan*>(plan));
    }
    auto g = std::make_unique<hbc_graph>();
    g->g = device_graph_create(plan->p, op, fields, nfields, reps, stream);
    *out = g.release();
  });
}

int hbc_graph_launch(hbc_graph* g, void* stream) {
  return guard([&] {
    need(g && g->g, "NULL graph");
    device_graph_launch(g->g, stream);
  });
}

void hbc_graph_destroy(hbc_graph* g) {
  if (!g) return;
  device_graph_destroy(g->g);
  delete g;
}

int hbc_consumer_create(const hbc_plan* plan, int32_t noffsets, const int64_t* offsets, const double* weights,
                        hbc_consumer** out) {
  hbc_consumer* c = nullptr;
  const int rc = guard([&] {
    need(plan != nullptr, "NULL plan");
    need(offsets && weights && out, "NULL argument");
    c = new hbc_consumer;
    c->plan = plan;
    compile_consumer(plan->p, noffsets, offsets, weights, c->host);
    // a host-only plan's consumer is compiled (stats) but never uploaded
    if (!(plan->p.flags & HBC_PLAN_HOST_ONLY)) c->dev = device_consumer_upload(plan->p, c->host);
    *out = c;
    c = nullptr;
  });
  if (c) {
    device_consumer_free(c->dev);
    delete c;
  }
  return rc;
}

int hbc_consumer_apply(const hbc_consumer* c, const void* x, int64_t x_nelem, void* y, int64_t y_nelem,
                       int32_t fused, void* stream) {
  return guard([&] {
    need(c != nullptr, "NULL consumer");
    check_device_plan(c->plan);
    check_field(x);
    check_field(y);
    check_size(c->plan, x_nelem);
    const int64_t want = c->host.ndata * c->plan->p.layout.inner;
    if (y_nelem != want)
      fail(HBC_EINVAL, "y has " + std::to_string(y_nelem) + " values, the consumer writes " + std::to_string(want));
    device_consumer_apply(c->plan->p, c->host, c->dev, x, y, fused != 0, stream);
  });
}

int hbc_consumer_stats(const hbc_consumer* c, int64_t* boundary_rows, int64_t* boundary_entries) {
  return guard([&] {
    need(c && boundary_rows && boundary_entries, "NULL argument");
    *boundary_rows = (int64_t)c->host.brow_y.size();
    *boundary_entries = (int64_t)c->host.bcol.size();
  });
}

void hbc_consumer_destroy(hbc_consumer* c) {
  if (!c) return;
  device_consumer_free(c->dev);
  delete c;
}

int hbc_stencil27(const hbc_plan* plan, const void* x, int64_t x_nelem, void* y, int64_t y_nelem, void* stream) {
  return guard([&] {
    check_device_plan(plan);
    check_field(x);
    check_field(y);
    check_stencil_sizes(plan, x_nelem, y_nelem);
    device_stencil27(const_cast<hbc_plan*>(plan)->p, x, y, stream, false, nullptr);
  });
}

int hbc_fused_stencil27(const hbc_plan* plan, void* x, int64_t x_nelem, void* y, int64_t y_nelem,
                        int32_t write_ghosts, void* stream) {
  return guard([&] {
    check_device_plan(plan);
    check_field(x);
    check_field(y);
    check_stencil_sizes(plan, x_nelem, y_nelem);
    device_stencil27(const_cast<hbc_plan*>(plan)->p, x, y, stream, true, write_ghosts ? x : nullptr);
  });
}

int hbc_cs_lagrange_weights(int64_t N, int64_t h, int32_t* base_dev, double* w_dev, void* stream) {
  return guard([&] {
    need(base_dev && w_dev, "NULL argument");
    need(N >= 4 && h >= 1 && 2 * h <= N,
         "cubed sphere needs N >= 4 and 1 <= h <= N/2 (deeper ghost layers leave the face's gnomonic chart)");
    device_cs_weights(N, h, base_dev, w_dev, stream);
  });
}

// ---- batch ----------------------------------------------------------------------------
int hbc_batch_create(hbc_plan* const* plans, int32_t n, hbc_batch** out) {
  return guard([&] {
    need(plans && out && n >= 1, "bad batch arguments");
    std::vector<Plan*> ps;
    for (int k = 0; k < n; ++k) {
      check_device_plan(plans[k]);
      ps.push_back(&plans[k]->p);
      need(plans[k]->p.dtype == plans[0]->p.dtype, "all plans of a batch need the same dtype");
      need(plans[k]->p.layout.order == HBC_POINT_MAJOR, "batches take point-major plans");
      if (plans[k]->p.stats.rows_data > 0) fail(HBC_EUNSUPPORTED, "batches do not take plans with data rows");
    }
    auto b = std::make_unique<hbc_batch>();
    b->plans.assign(ps.begin(), ps.end());
    b->b = device_batch_create(ps.data(), n);
    *out = b.release();
  });
}

void hbc_batch_destroy(hbc_batch* b) {
  if (!b) return;
  device_batch_destroy(b->b);
  delete b;
}

int hbc_batch_bind(hbc_batch* b, void* const* fields, const int64_t* nelem) {
  return guard([&] {
    need(b && fields && nelem, "NULL argument");
    const int n = (int)b->plans.size();
    for (int k = 0; k < n; ++k) {
      const Plan& p = *b->plans[k];
      need(nelem[k] == p.grid.ncells * p.layout.inner, "batch field size does not match its plan");
    }
    device_batch_bind(b->b, fields);
  });
}

int hbc_batch_apply(hbc_batch* b, void* stream) {
  return guard([&] {
    need(b != nullptr, "NULL argument");
    device_batch_apply(b->b, stream);
  });
}

int hbc_batch_graph_capture(hbc_batch* b, void* stream) {
  return guard([&] {
    need(b != nullptr, "NULL argument");
    device_batch_capture(b->b, stream);
  });
}

int hbc_batch_graph_launch(hbc_batch* b, void* stream) {
  return guard([&] {
    need(b != nullptr, "NULL argument");
    device_batch_launch_graph(b->b, stream);
  });
}

int hbc_batch_get_tune(const hbc_batch* b, hbc_tune* out) {
  return guard([&] {
    need(b && out, "NULL argument");
    *out = device_batch_get_tune(b->b);
  });
}

int hbc_batch_set_tune(hbc_batch* b, const hbc_tune* t) {
  return guard([&] {
    need(b && t, "NULL argument");
    device_batch_set_tune(b->b, *t);
  });
}

int hbc_batch_autotune(hbc_batch* b, const char* cache_path, void* stream, double* ms) {
  return guard([&] {
    need(b != nullptr, "NULL argument");
    double t = device_batch_autotune(b->b, cache_path, stream);
    if (ms) *ms = t;
  });
}

int hbc_batch_stats(const hbc_batch* b, hbc_stats* out) {
  return guard([&] {
    need(b && out, "NULL argument");
    device_batch_stats(b->b, out);
  });
}

}  // extern "C"
