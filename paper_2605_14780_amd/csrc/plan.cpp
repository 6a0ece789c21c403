// Host plan compiler: program of basic sub-matrices -> disjoint row boxes ->
// device segment / ELL / CSR / b / adjoint tables and a tile list.
//
// Sec. IV-B turns overlapping validity predicates into a non-overlapping set
// whose members each imply or exclude every original predicate; Sec. IV-C then
// splits the iteration space into disjoint convex pieces that run
// independently.  Here every validity set is a box, so both steps are integer
// box arithmetic: a box refinement yields pieces that each carry the list of
// sub-matrices / sub-vectors covering them, and each piece becomes one
// segment (a box with one kind of row).
#include <algorithm>
#include <climits>
#include <cstring>
#include <map>
#include <numeric>
#include <unordered_map>

#include "hbc_internal.hpp"

namespace hbc {

// ---- boxes --------------------------------------------------------------------
bool intersects(const Box& a, const Box& b) {
  for (int d = 0; d < a.nd; ++d)
    if (std::max(a.lo[d], b.lo[d]) >= std::min(a.hi[d], b.hi[d])) return false;
  return true;
}

Box intersect(const Box& a, const Box& b) {
  Box r = a;
  for (int d = 0; d < a.nd; ++d) {
    r.lo[d] = std::max(a.lo[d], b.lo[d]);
    r.hi[d] = std::min(a.hi[d], b.hi[d]);
  }
  return r;
}

std::vector<Box> subtract(const Box& a, const Box& b) {
  std::vector<Box> out;
  if (!intersects(a, b)) {
    out.push_back(a);
    return out;
  }
  Box cur = a;
  for (int d = 0; d < a.nd; ++d) {
    if (cur.lo[d] < b.lo[d]) {
      Box p = cur;
      p.hi[d] = b.lo[d];
      out.push_back(p);
      cur.lo[d] = b.lo[d];
    }
    if (cur.hi[d] > b.hi[d]) {
      Box p = cur;
      p.lo[d] = b.hi[d];
      out.push_back(p);
      cur.hi[d] = b.hi[d];
    }
  }
  return out;
}

// ---- grid ---------------------------------------------------------------------
int Grid::owner(const int64_t* c) const {
  for (size_t b = 0; b < blocks.size(); ++b)
    if (blocks[b].full.contains(c)) return (int)b;
  return -1;
}

int64_t Grid::cell(int b, const int64_t* c) const {
  const Block& B = blocks[b];
  int64_t off = B.first_cell;
  for (int d = 0; d < nd; ++d) off += (c[d] - B.full.lo[d]) * B.stride[d];
  return off;
}

bool Grid::unlinear(int64_t lin, int64_t* c) const {
  if (lin < 0) return false;
  for (int d = nd - 1; d >= 0; --d) {
    int64_t e = hi[d] - lo[d];
    c[d] = lo[d] + lin % e;
    lin /= e;
  }
  return lin == 0;
}

int64_t Grid::ghost_cells() const {
  int64_t n = 0;
  for (const Block& b : blocks) n += b.full.count() - b.data.count();
  return n;
}

// ---- rotation codes ---------------------------------------------------------------
int rot_code(const int32_t* R) {
  if (!R) return 0;
  int32_t a = R[0], b = R[1], c = R[2], d = R[3];
  auto unit = [](int32_t v) { return v == 1 || v == -1; };
  if (unit(a) && b == 0 && c == 0 && unit(d)) return (a < 0 ? 2 : 0) | (d < 0 ? 4 : 0);
  if (a == 0 && unit(b) && unit(c) && d == 0) return 1 | (b < 0 ? 2 : 0) | (c < 0 ? 4 : 0);
  return -1;
}

int rot_inverse(int code) {
  if (!(code & 1)) return code;
  int s0 = (code >> 1) & 1, s1 = (code >> 2) & 1;
  return 1 | (s1 << 1) | (s0 << 2);
}

void rot_matrix(int code, int32_t* R) {
  int s0 = (code & 2) ? -1 : 1, s1 = (code & 4) ? -1 : 1;
  if (code & 1) {
    R[0] = 0; R[1] = s0; R[2] = s1; R[3] = 0;
  } else {
    R[0] = s0; R[1] = 0; R[2] = 0; R[3] = s1;
  }
}

// ---- compilation --------------------------------------------------------------------
namespace {

struct Piece {
  Box box;
  std::vector<int> covers;  // sub indices (matrix and vector subs)
};

// Row-major linear index of multi-index c inside box b.
int64_t box_linear(const Box& b, const int64_t* c) {
  int64_t k = 0;
  for (int d = 0; d < b.nd; ++d) k = k * (b.hi[d] - b.lo[d]) + (c[d] - b.lo[d]);
  return k;
}

// Iterate the multi-indices of a box in row-major order.
template <class F>
void for_box(const Box& b, F&& f) {
  int64_t c[HBC_MAX_DIM];
  for (int d = 0; d < b.nd; ++d) c[d] = b.lo[d];
  int64_t n = b.count();
  for (int64_t k = 0; k < n; ++k) {
    f(c, k);
    for (int d = b.nd - 1; d >= 0; --d) {
      if (++c[d] < b.hi[d]) break;
      c[d] = b.lo[d];
    }
  }
}

// Iterate the multi-indices of a box with the dims in `order` (slowest first);
// dims not listed stay at their lower bound (extent 1).
template <class F>
void for_box_order(const Box& b, const std::vector<int>& order, F&& f) {
  int64_t c[HBC_MAX_DIM];
  for (int d = 0; d < b.nd; ++d) c[d] = b.lo[d];
  const int64_t n = b.count();
  const int k = (int)order.size();
  for (int64_t q = 0; q < n; ++q) {
    f(c, q);
    for (int j = k - 1; j >= 0; --j) {
      const int d = order[j];
      if (++c[d] < b.hi[d]) break;
      c[d] = b.lo[d];
    }
  }
}

// Data cell of a global linear index; HBC_ERANGE if it is not a data cell.
int64_t data_cell_of_linear(const Grid& g, int64_t lin) {
  int64_t c[HBC_MAX_DIM];
  if (!g.unlinear(lin, c)) fail(HBC_ERANGE, "column index " + std::to_string(lin) + " is outside the global box");
  int b = g.owner(c);
  if (b < 0 || !g.blocks[b].data.contains(c))
    fail(HBC_ERANGE, "column index " + std::to_string(lin) + " is not a data cell");
  return g.cell(b, c);
}

void map_apply(const Sub& s, int nd, const int64_t* r, int64_t* out) {
  for (int e = 0; e < nd; ++e) {
    int64_t v = s.off[e];
    for (int d = 0; d < nd; ++d) v += s.M[e * nd + d] * r[d];
    out[e] = v;
  }
}

// Refine boxes so that pieces are disjoint and each lies fully inside or
// outside every sub's box (the non-overlapping set of Sec. IV-B).
std::vector<Piece> refine(const std::vector<Sub>& subs) {
  std::vector<Piece> P;
  for (int s = 0; s < (int)subs.size(); ++s) {
    const Box& S = subs[s].rows;
    std::vector<Piece> next;
    std::vector<Box> rest{S};
    for (Piece& p : P) {
      if (p.box.nd == 0 || !intersects(p.box, S)) {
        next.push_back(std::move(p));
        continue;
      }
      Piece in{intersect(p.box, S), p.covers};
      in.covers.push_back(s);
      next.push_back(in);
      for (const Box& o : subtract(p.box, S)) next.push_back(Piece{o, p.covers});
      std::vector<Box> r2;
      for (const Box& r : rest)
        for (const Box& o : subtract(r, p.box)) r2.push_back(o);
      rest.swap(r2);
    }
    for (const Box& r : rest) next.push_back(Piece{r, {s}});
    P.swap(next);
  }
  return P;
}

}  // namespace

// Closed components of the data rows: rows are joined when one reads a cell
// another writes.  Every written cell a component reads is then written by
// that component, so reading all its columns first and writing its rows after
// gives the input-field semantics without scratch.  Used when every
// component has at most DC_MAX rows, columns and entries per row.
static void build_data_components(HostTables& T) {
  T.dc_ok = false;
  T.dc_comp.clear();
  T.dc_row_dst.clear();
  T.dc_row_ent.clear();
  T.dc_row_n.clear();
  T.dc_slot.clear();
  T.dc_w.clear();
  const int64_t n = (int64_t)T.dr_cell.size();
  if (n == 0) return;
  std::unordered_map<int32_t, int64_t> row_of;
  for (int64_t r = 0; r < n; ++r) row_of[T.dr_cell[r]] = r;
  std::vector<int64_t> parent(n);
  std::iota(parent.begin(), parent.end(), 0);
  auto find = [&](int64_t a) {
    while (parent[a] != a) a = parent[a] = parent[parent[a]];
    return a;
  };
  for (int64_t r = 0; r < n; ++r)
    for (int64_t e = T.dr_ptr[r]; e < T.dr_ptr[r + 1]; ++e) {
      auto it = row_of.find(T.dr_col[e]);
      if (it == row_of.end()) continue;
      const int64_t a = find(r), b = find(it->second);
      if (a != b) parent[std::max(a, b)] = std::min(a, b);
    }
  std::map<int64_t, std::vector<int64_t>> comps;  // root -> rows (ascending)
  for (int64_t r = 0; r < n; ++r) comps[find(r)].push_back(r);
  for (const auto& kv : comps) {
    const std::vector<int64_t>& rows = kv.second;
    DataComp c{};
    c.first_row = (int32_t)T.dc_row_dst.size();
    c.nrow = (int32_t)rows.size();
    if (c.nrow > DC_MAX) return;
    for (int64_t r : rows) {
      if (T.dr_ptr[r + 1] - T.dr_ptr[r] > DC_MAX) return;
      T.dc_row_dst.push_back(T.dr_cell[r]);
      T.dc_row_ent.push_back((int32_t)T.dc_slot.size());
      T.dc_row_n.push_back((int32_t)(T.dr_ptr[r + 1] - T.dr_ptr[r]));
      for (int64_t e = T.dr_ptr[r]; e < T.dr_ptr[r + 1]; ++e) {
        int slot = -1;
        for (int m = 0; m < c.ncol; ++m)
          if (c.col[m] == T.dr_col[e]) slot = m;
        if (slot < 0) {
          if (c.ncol == DC_MAX) return;
          slot = c.ncol++;
          c.col[slot] = T.dr_col[e];
        }
        T.dc_slot.push_back(slot);
        T.dc_w.push_back(T.dr_val[e]);
      }
    }
    T.dc_comp.push_back(c);
  }
  T.dc_ok = true;
}

// b values of one segment (Sec. III-B: the affine part of F, the sum of the
// sub-vectors that cover a row)
static void fill_bseg(const BSeg& bs, const std::vector<Sub>& vsubs, std::vector<double>& bval) {
  for_box_order(bs.box, bs.order, [&](const int64_t* r, int64_t q) {
    for (int64_t l = 0; l < bs.bi; ++l) {
      double acc = 0.0;
      bool first = true;
      for (int v : bs.vecs) {
        const Sub& s = vsubs[v];
        const int64_t k = box_linear(s.rows, r);
        const double x = s.b[k * s.ninner + (s.ninner == 1 ? 0 : l)];
        acc = first ? x : acc + x;
        first = false;
      }
      bval[bs.brow + q * bs.bi + l] = acc;
    }
  });
}

std::pair<int64_t, int64_t> plan_set_vector(Plan& plan, int32_t sub_id, const double* values) {
  int k = -1;
  for (size_t j = 0; j < plan.vsub_id.size(); ++j)
    if (plan.vsub_id[j] == sub_id) k = (int)j;
  if (k < 0) fail(HBC_EINVAL, "sub_id " + std::to_string(sub_id) + " is not a sub-vector of the plan's program");
  Sub& s = plan.vsubs[k];
  if (!values && !s.b.empty()) fail(HBC_EINVAL, "NULL values");
  std::copy(values, values + s.b.size(), s.b.begin());
  int64_t first = INT64_MAX, last = 0;
  for (const BSeg& bs : plan.bsegs) {
    if (std::find(bs.vecs.begin(), bs.vecs.end(), k) == bs.vecs.end()) continue;
    fill_bseg(bs, plan.vsubs, plan.host.bval);
    first = std::min(first, bs.brow);
    last = std::max(last, bs.brow + bs.box.count() * bs.bi);
  }
  if (first >= last) return {0, 0};
  return {first, last};
}

void compile_plan(const Program& prog, const Layout& lay, int dtype, Plan& plan) {
  const Grid& g = prog.grid;
  plan.grid = g;
  plan.layout = lay;
  plan.dtype = dtype;
  if (lay.inner < 1) fail(HBC_EINVAL, "layout.inner must be >= 1");
  if (lay.order != HBC_POINT_MAJOR && lay.order != HBC_PLANE_MAJOR) fail(HBC_EINVAL, "bad layout order");
  if (lay.vec_len < 0 || (lay.vec_len > 0 && (lay.vec_lo < 0 || lay.vec_stride < lay.vec_len ||
                                               lay.vec_lo + lay.vec_stride + lay.vec_len > lay.inner)))
    fail(HBC_EINVAL, "vector slots do not fit the inner extent");
  if (g.ncells >= (int64_t(1) << 31) - 1) fail(HBC_EUNSUPPORTED, "more than 2^31-2 cells per plan");
  if (g.blocks.empty()) fail(HBC_EINVAL, "grid has no blocks");

  // 1. validate rows; expand the zero-rest subs; keep the sub-vectors
  //    (their values can be replaced after compile, plan_set_vector)
  std::vector<Sub> subs;
  std::vector<int> vsub_of;  // per entry of subs: its index in plan.vsubs, or -1
  std::vector<int> zero_rest_blocks;
  plan.vsubs.clear();
  plan.vsub_id.clear();
  plan.bsegs.clear();
  for (size_t id = 0; id < prog.subs.size(); ++id) {
    const Sub& s0 = prog.subs[id];
    int vk = -1;
    if (s0.kind == SUB_VEC) {
      vk = (int)plan.vsubs.size();
      plan.vsubs.push_back(s0);
      plan.vsub_id.push_back((int32_t)id);
    }
    if (s0.kind == SUB_ZERO_REST) {
      zero_rest_blocks.push_back(s0.block);
      continue;
    }
    if (s0.rows.empty()) continue;
    Sub s = s0;
    int b = g.owner(s.rows.lo);
    if (b < 0 || !g.blocks[b].full.contains(s.rows))
      fail(HBC_ERANGE, "sub-matrix rows do not lie in one block's full region");
    if (intersects(s.rows, g.blocks[b].data))
      fail(HBC_ERANGE, "sub-matrix rows include data cells (only ghost rows are written)");
    s.block = b;
    subs.push_back(std::move(s));
    vsub_of.push_back(vk);
  }
  for (int b : zero_rest_blocks) {
    if (b < 0 || b >= (int)g.blocks.size()) fail(HBC_EINVAL, "zero-rest block out of range");
    std::vector<Box> rest = subtract(g.blocks[b].full, g.blocks[b].data);
    for (const Sub& s : subs) {
      if (s.block != b || s.kind == SUB_VEC) continue;
      std::vector<Box> r2;
      for (const Box& r : rest)
        for (const Box& o : subtract(r, s.rows)) r2.push_back(o);
      rest.swap(r2);
    }
    for (const Box& r : rest) {
      if (r.empty()) continue;
      Sub z;
      z.kind = SUB_ZERO;
      z.rows = r;
      z.block = b;
      subs.push_back(z);
      vsub_of.push_back(-1);
    }
  }

  // 2. overlap rule (R2): sub-matrices are pairwise disjoint, sub-vectors too,
  //    unless the program allows summing.
  const bool allow_sum = prog.flags & HBC_ALLOW_OVERLAP_SUM;
  for (size_t a = 0; a < subs.size(); ++a)
    for (size_t c = a + 1; c < subs.size(); ++c) {
      bool va = subs[a].kind == SUB_VEC, vc = subs[c].kind == SUB_VEC;
      if (va != vc || subs[a].block != subs[c].block) continue;
      if (!allow_sum && intersects(subs[a].rows, subs[c].rows))
        fail(HBC_EOVERLAP, std::string("overlapping ") + (va ? "sub-vector" : "sub-matrix") + " rows (subs " +
                               std::to_string(a) + " and " + std::to_string(c) + ")");
    }

  // 3. pieces
  std::vector<Piece> pieces = refine(subs);
  // 3a. consumer footprint (Sec. IV-C): keep only the parts of the pieces that
  //     some consumer read reaches; live ghost region of a block = union over
  //     offsets of (data + offset) inside the full box, minus the data box
  int64_t dead = 0, live_ghosts = 0;
  if (!prog.consumer.empty()) {
    const size_t no = prog.consumer.size() / g.nd;
    std::vector<std::vector<Box>> live(g.blocks.size());
    for (size_t b = 0; b < g.blocks.size(); ++b) {
      const Block& B = g.blocks[b];
      std::vector<Box> L;  // disjoint
      for (size_t o = 0; o < no; ++o) {
        Box sh = B.data;
        for (int d = 0; d < g.nd; ++d) {
          sh.lo[d] += prog.consumer[o * g.nd + d];
          sh.hi[d] += prog.consumer[o * g.nd + d];
        }
        if (!intersects(sh, B.full)) continue;
        std::vector<Box> add = subtract(intersect(sh, B.full), B.data);
        for (const Box& have : L) {  // keep L disjoint
          std::vector<Box> a2;
          for (const Box& a : add)
            for (const Box& x : subtract(a, have)) a2.push_back(x);
          add.swap(a2);
        }
        for (const Box& a : add)
          if (!a.empty()) L.push_back(a);
      }
      for (const Box& a : L) live_ghosts += a.count();
      live[b].swap(L);
    }
    std::vector<Piece> kept;
    for (const Piece& pc : pieces) {
      const int b = subs[pc.covers[0]].block;
      int64_t in = 0;
      for (const Box& a : live[b]) {
        if (!intersects(pc.box, a)) continue;
        Piece q{intersect(pc.box, a), pc.covers};
        in += q.box.count();
        kept.push_back(std::move(q));
      }
      dead += pc.box.count() - in;
    }
    pieces.swap(kept);
  } else {
    live_ghosts = g.ghost_cells();
  }
  // deterministic order: by block, then by origin
  std::sort(pieces.begin(), pieces.end(), [&](const Piece& x, const Piece& y) {
    int bx = subs[x.covers[0]].block, by = subs[y.covers[0]].block;
    if (bx != by) return bx < by;
    return std::lexicographical_compare(x.box.lo, x.box.lo + x.box.nd, y.box.lo, y.box.lo + y.box.nd);
  });

  HostTables& T = plan.host;
  hbc_stats& st = plan.stats;
  std::memset(&st, 0, sizeof(st));
  std::vector<int64_t> sources;
  const int nd = g.nd;
  int64_t row_base = 0;

  for (const Piece& pc : pieces) {
    std::vector<int> mats, vecs;
    for (int s : pc.covers) (subs[s].kind == SUB_VEC ? vecs : mats).push_back(s);
    const int b = subs[pc.covers[0]].block;
    const Block& B = g.blocks[b];
    DevSeg seg;
    std::memset(&seg, 0, sizeof(seg));
    seg.nrows = pc.box.count();
    seg.row_base = row_base;
    row_base += seg.nrows;
    seg.w = 1.0;
    // full-dimension strides before dropping extent-1 dims
    int64_t dst_st[HBC_MAX_DIM], src_st[HBC_MAX_DIM] = {0};
    for (int d = 0; d < nd; ++d) dst_st[d] = B.stride[d];
    seg.dst_base = g.cell(b, pc.box.lo);
    int rot = 0;
    if (!mats.empty()) {
      rot = subs[mats[0]].rot;
      for (int m : mats)
        if (subs[m].rot != rot) fail(HBC_EOVERLAP, "overlapping rows with different component rotations");
    }
    seg.rot = rot;
    // device row order: the box's non-trivial dims; for table rows of
    // point-major fields the longest dim goes fastest, so that consecutive rows
    // of a run share source cells (a face-edge strip walks along the edge)
    std::vector<int> order;
    for (int d = 0; d < nd; ++d)
      if (pc.box.extent(d) > 1) order.push_back(d);
    const bool table_rows = !mats.empty() && !(mats.size() == 1 && (subs[mats[0]].kind == SUB_MAP ||
                                                                     subs[mats[0]].kind == SUB_ZERO));
#ifndef HBC_NATURAL_ROW_ORDER
    if (table_rows && lay.order == HBC_POINT_MAJOR)
#else
    if (false)
#endif
      std::stable_sort(order.begin(), order.end(),
                       [&](int a, int c) { return pc.box.extent(a) < pc.box.extent(c); });

    if (mats.size() == 1 && subs[mats[0]].kind == SUB_MAP) {
      const Sub& s = subs[mats[0]];
      seg.kind = SEG_MAP;
      seg.w = s.w;
      // the affine image of the piece: check its corners
      int sb = -1;
      for (int corner = 0; corner < (1 << nd); ++corner) {
        int64_t r[HBC_MAX_DIM], c[HBC_MAX_DIM];
        for (int d = 0; d < nd; ++d) r[d] = (corner >> d & 1) ? pc.box.hi[d] - 1 : pc.box.lo[d];
        map_apply(s, nd, r, c);
        int ob = g.owner(c);
        if (ob < 0 || !g.blocks[ob].data.contains(c) || (sb >= 0 && ob != sb))
          fail(HBC_ERANGE, "map sends rows outside one block's data region");
        sb = ob;
      }
      int64_t c0[HBC_MAX_DIM];
      map_apply(s, nd, pc.box.lo, c0);
      seg.src_base = g.cell(sb, c0);
      for (int d = 0; d < nd; ++d) {
        int64_t v = 0;
        for (int e = 0; e < nd; ++e) v += s.M[e * nd + d] * g.blocks[sb].stride[e];
        src_st[d] = v;
      }
      st.rows_map += seg.nrows;
      st.nnz += seg.nrows;
      for_box_order(pc.box, order, [&](const int64_t* r, int64_t) {
        int64_t c[HBC_MAX_DIM];
        map_apply(s, nd, r, c);
        sources.push_back(g.cell(sb, c));
      });
    } else if (mats.size() == 1 && subs[mats[0]].kind == SUB_ZERO) {
      seg.kind = SEG_ZERO;
      st.rows_zero += seg.nrows;
    } else if (mats.size() == 1 && subs[mats[0]].kind == SUB_ELL) {
      const Sub& s = subs[mats[0]];
      seg.kind = SEG_ELL;
      seg.width = s.width;
      // absolute element offset: rows of this segment start here (width entries each)
      seg.tab = (int64_t)T.ell_col.size();
      for_box_order(pc.box, order, [&](const int64_t* r, int64_t) {
        int64_t k = box_linear(s.rows, r);
        for (int m = 0; m < s.width; ++m) {
          int64_t lin = s.cols[k * s.width + m];
          double v = s.vals[k * s.width + m];
          if (lin < 0) {
            T.ell_col.push_back(-1);
            T.ell_val.push_back(0.0);
            seg.flags |= SEGF_ELL_PADDED;
            continue;
          }
          int64_t cell = data_cell_of_linear(g, lin);
          T.ell_col.push_back((int32_t)cell);
          T.ell_val.push_back(v);
          sources.push_back(cell);
          st.nnz += 1;
        }
      });
      st.rows_ell += seg.nrows;
    } else if (!mats.empty()) {
      // one CSR sub, or several overlapping subs summed into merged CSR rows
      seg.kind = SEG_CSR;
      seg.tab = (int64_t)T.csr_ptr.size();
      for_box_order(pc.box, order, [&](const int64_t* r, int64_t) {
        std::vector<std::pair<int64_t, double>> ents;
        for (int m : mats) {
          const Sub& s = subs[m];
          if (s.kind == SUB_MAP) {
            int64_t c[HBC_MAX_DIM];
            map_apply(s, nd, r, c);
            int ob = g.owner(c);
            if (ob < 0 || !g.blocks[ob].data.contains(c)) fail(HBC_ERANGE, "map sends a row outside the data region");
            ents.emplace_back(g.cell(ob, c), s.w);
          } else if (s.kind == SUB_ELL) {
            int64_t k = box_linear(s.rows, r);
            for (int q = 0; q < s.width; ++q)
              if (s.cols[k * s.width + q] >= 0)
                ents.emplace_back(data_cell_of_linear(g, s.cols[k * s.width + q]), s.vals[k * s.width + q]);
          } else if (s.kind == SUB_CSR) {
            int64_t k = box_linear(s.rows, r);
            for (int64_t q = s.ptr[k]; q < s.ptr[k + 1]; ++q)
              ents.emplace_back(data_cell_of_linear(g, s.cols[q]), s.vals[q]);
          }
        }
        if (mats.size() > 1) {  // sum duplicate columns
          std::stable_sort(ents.begin(), ents.end(),
                           [](const auto& x, const auto& y) { return x.first < y.first; });
          std::vector<std::pair<int64_t, double>> m2;
          for (auto& e : ents) {
            if (!m2.empty() && m2.back().first == e.first)
              m2.back().second += e.second;
            else
              m2.push_back(e);
          }
          ents.swap(m2);
        }
        T.csr_ptr.push_back((int64_t)T.csr_col.size());
        for (auto& e : ents) {
          T.csr_col.push_back((int32_t)e.first);
          T.csr_val.push_back(e.second);
          sources.push_back(e.first);
        }
        st.nnz += (int64_t)ents.size();
      });
      T.csr_ptr.push_back((int64_t)T.csr_col.size());  // end of this segment's rows
      st.rows_csr += seg.nrows;
    } else {
      seg.kind = SEG_VEC;
      st.rows_vector_only += seg.nrows;
    }

    if (!vecs.empty()) {
      int64_t bi = 1;
      for (int v : vecs) bi = std::max(bi, subs[v].ninner);
      for (int v : vecs)
        if (subs[v].ninner != 1 && subs[v].ninner != lay.inner)
          fail(HBC_EINVAL, "sub-vector inner width must be 1 or layout.inner");
      seg.has_b = 1;
      seg.b_inner = (int32_t)bi;
      seg.brow = (int64_t)T.bval.size();
      BSeg bs;
      bs.box = pc.box;
      bs.order = order;
      for (int v : vecs) bs.vecs.push_back(vsub_of[v]);
      bs.bi = bi;
      bs.brow = seg.brow;
      T.bval.resize((size_t)(seg.brow + seg.nrows * bi));
      fill_bseg(bs, plan.vsubs, T.bval);
      plan.bsegs.push_back(std::move(bs));
      st.rows_with_b += seg.nrows;
    }

    // drop extent-1 dims, then merge dims contiguous in both dst and src
    int k = 0;
    int64_t ext[HBC_MAX_DIM], ds[HBC_MAX_DIM], ss[HBC_MAX_DIM];
    for (int d : order) {
      ext[k] = pc.box.extent(d);
      ds[k] = dst_st[d];
      ss[k] = src_st[d];
      ++k;
    }
    if (k == 0) {
      ext[0] = 1; ds[0] = 1; ss[0] = 0; k = 1;
    }
    int m = 0;
    for (int d = 1; d < k; ++d) {
      bool merge = ds[m] == ext[d] * ds[d] && (seg.kind != SEG_MAP || ss[m] == ext[d] * ss[d]);
      if (merge) {
        ext[m] *= ext[d];
        ds[m] = ds[d];
        ss[m] = ss[d];
      } else {
        ++m;
        ext[m] = ext[d]; ds[m] = ds[d]; ss[m] = ss[d];
      }
    }
    k = m + 1;
    if (k > SEG_MAXD) fail(HBC_EUNSUPPORTED, "row box has more than 4 non-trivial dimensions");
    seg.nd = k;
    for (int d = 0; d < SEG_MAXD; ++d) {
      seg.ext[d] = d < k ? (int32_t)ext[d] : 1;
      seg.dst_stride[d] = d < k ? ds[d] : 0;
      seg.src_stride[d] = d < k ? ss[d] : 0;
      if (d < k && ext[d] >= (int64_t(1) << 31)) fail(HBC_EUNSUPPORTED, "box extent too large");
    }
    T.segs.push_back(seg);
    T.seg_box.push_back(pc.box);
    T.seg_order.push_back(order);
    // per-row destination (and MAP source) cells in device order
    {
      int64_t c[SEG_MAXD] = {0};
      for (int64_t r = 0; r < seg.nrows; ++r) {
        int64_t q = r, dst = seg.dst_base, src = seg.src_base;
        for (int d = seg.nd - 1; d >= 0; --d) {
          c[d] = q % seg.ext[d];
          q /= seg.ext[d];
          dst += c[d] * seg.dst_stride[d];
          src += c[d] * seg.src_stride[d];
        }
        T.row_dst.push_back((int32_t)dst);
        T.row_src.push_back(seg.kind == SEG_MAP ? (int32_t)src : 0);
      }
    }
  }

  // 3b. data rows (block-edge averaging): validated like the ghost rows, but
  //     inside a data region; staged through scratch by the apply
  for (size_t a = 0; a < prog.dsubs.size(); ++a) {
    const DataSub& ds = prog.dsubs[a];
    if (ds.rows.empty()) continue;
    int b = g.owner(ds.rows.lo);
    if (b < 0 || !g.blocks[b].data.contains(ds.rows))
      fail(HBC_ERANGE, "data-row box does not lie in one block's data region");
    for (size_t c = a + 1; c < prog.dsubs.size(); ++c)
      if (intersects(ds.rows, prog.dsubs[c].rows)) fail(HBC_EOVERLAP, "overlapping data-row boxes");
    for_box(ds.rows, [&](const int64_t* r, int64_t k) {
      T.dr_cell.push_back((int32_t)g.cell(b, r));
      T.dr_ptr.push_back((int64_t)T.dr_col.size());
      for (int64_t e = ds.ptr[k]; e < ds.ptr[k + 1]; ++e) {
        const int64_t cell = data_cell_of_linear(g, ds.cols[e]);
        T.dr_col.push_back((int32_t)cell);
        T.dr_val.push_back(ds.vals[e]);
        sources.push_back(cell);
        st.nnz++;
      }
    });
  }
  T.dr_ptr.push_back((int64_t)T.dr_col.size());
  st.rows_data = (int64_t)T.dr_cell.size();
  build_data_components(T);
  if (st.rows_data > 0 && lay.order != HBC_POINT_MAJOR)
    fail(HBC_EUNSUPPORTED, "data rows need the point-major layout");

  // 4. statistics
  st.ghost_cells = g.ghost_cells();
  st.rows_covered = row_base;
  st.rows_uncovered = st.ghost_cells - st.rows_covered;
  st.rows_dead = dead;
  st.ghost_cells_live = live_ghosts;
  if ((prog.flags & HBC_STRICT_COVER) && live_ghosts - st.rows_covered > 0)
    fail(HBC_EUNCOVERED, std::to_string(live_ghosts - st.rows_covered) + " ghost cells are covered by no sub-matrix");
  std::sort(sources.begin(), sources.end());
  st.unique_sources = (int64_t)(std::unique(sources.begin(), sources.end()) - sources.begin());
  st.segments = (int64_t)T.segs.size();
  st.ghost_values = st.rows_covered * lay.inner;
  const double es = dtype == HBC_F64 ? 8.0 : 4.0;
  const double I = (double)lay.inner;
  double tables = (double)T.ell_col.size() * (4.0 + es) + (double)T.csr_col.size() * (4.0 + es) +
                  (double)T.csr_ptr.size() * 8.0 + (double)T.bval.size() * es +
                  (double)T.dr_col.size() * (4.0 + es) + (double)T.dr_cell.size() * 12.0;
  st.alg_bytes = es * I * (double)(st.rows_covered + st.rows_data + st.unique_sources) + tables;
  // adjoint: read + zero the covered ghosts, read-modify-write the sources,
  // one (ghost, weight, rotation) entry per nonzero and a pointer per source
  st.alg_bytes_adjoint = es * I * (2.0 * (double)st.rows_covered + 2.0 * (double)st.unique_sources) +
                         (double)st.nnz * (8.0 + es + 4.0) + (double)st.unique_sources * 16.0;

  // 5. launch shape and tiles
  plan.vec = 1;
  if (lay.order == HBC_POINT_MAJOR) {
    int v = dtype == HBC_F64 ? 2 : 4;
    while (v > 1) {
      bool ok = lay.inner % v == 0 && (lay.vec_len == 0 || (lay.vec_lo % v == 0 && lay.vec_stride % v == 0 &&
                                                             lay.vec_len % v == 0));
      if (ok) break;
      v /= 2;
    }
    plan.vec = v;
    const int64_t nvec = lay.inner / v;
    int u = 16 / (v * (int)es);
    while (u > 1 && u > nvec) u /= 2;
    plan.unroll = u;
  }
  plan.tune = default_tune(plan);
  build_tiles(plan, plan.tune);
  compute_stencil_info(plan);
}

static int64_t pow2_ceil(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Whether a segment can take sliding windows, its column pattern aside: a
// 4-wide ELL segment without padding; with b values only from WIN_MIN_BYTES_B
// per row (the b loads of a run cost more than the window saves on shorter
// rows).
static bool win_seg_shape(const Plan& plan, const DevSeg& sg) {
  const int64_t es = plan.dtype == HBC_F64 ? 8 : 4;
  if (sg.kind != SEG_ELL || sg.width != 4 || (sg.flags & SEGF_ELL_PADDED) || sg.nrows == 0) return false;
  return !(sg.has_b && plan.layout.inner * es < WIN_MIN_BYTES_B);
}

// Whether build_windows can take a segment of the plan (its column patterns
// aside): point-major, whole 16-byte vectors, rows of >= WIN_MIN_BYTES, a
// segment of the window shape.
bool windows_possible(const Plan& plan) {
  const Layout& L = plan.layout;
  const int64_t es = plan.dtype == HBC_F64 ? 8 : 4;
  if (L.order != HBC_POINT_MAJOR || (plan.flags & HBC_PLAN_NO_WINDOWS) || plan.stats.rows_data > 0) return false;
  if (plan.vec * es != 16 || L.inner * es < WIN_MIN_BYTES) return false;
  if (L.inner * es >= (int64_t(1) << 31)) return false;  // a row is one 32-bit buffer range
  for (const DevSeg& sg : plan.host.segs)
    if (win_seg_shape(plan, sg)) return true;
  return false;
}

hbc_tune default_tune(const Plan& plan) {
  hbc_tune t{};
  t.block = 256;
  t.persistent = 0;
  t.window_order = 0;
  const int64_t rows = std::max<int64_t>(1, plan.stats.rows_covered);
  if (plan.layout.order == HBC_POINT_MAJOR) {
    // 16 bytes per lane (vec elements, unroll times): a row group covers a whole row
    int64_t nvec = plan.layout.inner / plan.vec;
    int64_t nacc = (nvec + plan.unroll - 1) / plan.unroll;
    t.lanes_per_row = (int32_t)std::min<int64_t>(t.block, pow2_ceil(nacc));
  } else {
    // plane-major: 8 planes per thread and batch, up to 16 thread sets over
    // the planes (16 consecutive rows per wavefront and plane)
    const int64_t sets = (plan.layout.inner + 7) / 8;
    t.lanes_per_row = (int32_t)std::min<int64_t>(16, pow2_ceil(sets));
  }
  const int64_t rows_per_pass = t.block / t.lanes_per_row;
  // Short tiles keep many workgroups in flight (the apply is latency bound per
  // row: table reads, then source loads, then stores): one batch of rows per
  // row group when groups take contiguous runs of rows, else about 4096 tiles
  // in all.
  int64_t rpt;
  if (plan.layout.order != HBC_POINT_MAJOR && t.lanes_per_row > 1) {
    rpt = rows_per_pass;  // one pass of rows over all planes per tile
  } else if (t.lanes_per_row >= CHUNK_LPR) {
    rpt = rows_per_pass * rows_per_batch(t.lanes_per_row);
  } else {
    rpt = std::max<int64_t>(rows / 4096, rows_per_pass);
    rpt = ((rpt + rows_per_pass - 1) / rows_per_pass) * rows_per_pass;
  }
  rpt = std::min<int64_t>(rpt, 16384);
  if (windows_possible(plan)) rpt = WIN_DEFAULT_ROWS;  // rows per sliding-window run
  t.rows_per_tile = (int32_t)rpt;
  return t;
}

// Segment rows in wide-tile order: the thinnest box dimension innermost, the
// others in box order (the last of equally thin dimensions is taken).
static std::vector<int64_t> wide_row_order(const DevSeg& sg) {
  const int nd = sg.nd;
  int thin = nd - 1;
  for (int k = 0; k < nd; ++k)
    if (sg.ext[k] < sg.ext[thin]) thin = k;
  std::vector<int> dims;
  for (int k = 0; k < nd; ++k)
    if (k != thin) dims.push_back(k);
  dims.push_back(thin);
  int64_t stride[SEG_MAXD];
  int64_t s = 1;
  for (int k = nd - 1; k >= 0; --k) {
    stride[k] = s;
    s *= sg.ext[k];
  }
  std::vector<int64_t> order((size_t)sg.nrows);
  int64_t idx[SEG_MAXD] = {0, 0, 0, 0};
  for (int64_t n = 0; n < sg.nrows; ++n) {
    int64_t r = 0;
    for (int k = 0; k < nd; ++k) r += idx[k] * stride[k];
    order[(size_t)n] = r;
    for (int q = nd - 1; q >= 0; --q) {  // advance the counter, dims[nd-1] fastest
      const int k = dims[(size_t)q];
      if (++idx[k] < sg.ext[k]) break;
      idx[k] = 0;
    }
  }
  return order;
}

// Wide-row tiles (see WideTile): the rows of a wide CSR segment in
// wide_row_order, cut greedily while their distinct source cells and entries
// fit.
static void build_wide(Plan& plan) {
  HostTables& T = plan.host;
  T.seg_wide.assign(T.segs.size(), 0);
  T.wtiles.clear();
  T.w_ucell.clear();
  T.w_row.clear();
  T.w_rp.clear();
  T.w_entw.clear();
  T.w_ents.clear();
  T.w_maxu = T.w_maxe = 0;
  plan.stats.rows_wide = plan.stats.wide_tiles = 0;
  if (plan.layout.order != HBC_POINT_MAJOR) return;
  const int64_t es = plan.dtype == HBC_F64 ? 8 : 4;
  if (plan.layout.inner * es < WIDE_ROW_BYTES || plan.layout.inner > (int64_t(1) << 30)) return;  // 32-bit slots
  std::unordered_map<int32_t, int32_t> local;
  for (size_t si = 0; si < T.segs.size(); ++si) {
    const DevSeg& sg = T.segs[si];
    if (sg.kind != SEG_CSR || sg.nrows == 0) continue;
    const int64_t nnz = T.csr_ptr[sg.tab + sg.nrows] - T.csr_ptr[sg.tab];
    if (nnz < WIDE_NNZ * sg.nrows) continue;
    bool fits = true;
    for (int64_t r = 0; r < sg.nrows && fits; ++r) {
      local.clear();
      for (int64_t e = T.csr_ptr[sg.tab + r]; e < T.csr_ptr[sg.tab + r + 1]; ++e) local[T.csr_col[e]] = 0;
      fits = (int64_t)local.size() <= WIDE_UCAP && T.csr_ptr[sg.tab + r + 1] - T.csr_ptr[sg.tab + r] <= WIDE_ECAP;
    }
    if (!fits) continue;
    T.seg_wide[si] = 1;
    const std::vector<int64_t> order = wide_row_order(sg);
    size_t n = 0;
    while (n < order.size()) {
      WideTile w{};
      w.rot = sg.rot;
      w.has_b = sg.has_b;
      w.b_inner = sg.b_inner;
      w.row_base = sg.row_base;
      w.brow = sg.brow;
      w.first_u = (int32_t)T.w_ucell.size();
      w.e0 = (int32_t)T.w_entw.size();
      w.r0 = (int32_t)T.w_row.size();
      w.rp0 = (int32_t)T.w_rp.size();
      T.w_rp.push_back(0);
      local.clear();
      while (n < order.size() && w.nrows < WIDE_ROWS) {
        const int64_t r = order[n];
        const int64_t b = T.csr_ptr[sg.tab + r], e = T.csr_ptr[sg.tab + r + 1];
        int add = 0;
        for (int64_t k = b; k < e; ++k)
          if (!local.count(T.csr_col[k])) ++add;  // repeats within the row count twice: conservative
        if (w.nu + add > WIDE_UCAP || w.ne + (e - b) > WIDE_ECAP) break;
        for (int64_t k = b; k < e; ++k) {
          auto it = local.find(T.csr_col[k]);
          if (it == local.end()) {
            it = local.emplace(T.csr_col[k], w.nu++).first;
            T.w_ucell.push_back(T.csr_col[k]);
          }
          T.w_entw.push_back(T.csr_val[k]);
          T.w_ents.push_back(it->second);
        }
        w.ne += (int32_t)(e - b);
        T.w_row.push_back((int32_t)r);
        T.w_rp.push_back(w.ne);
        ++w.nrows;
        ++n;
      }
      T.w_maxu = std::max(T.w_maxu, w.nu);
      T.w_maxe = std::max(T.w_maxe, w.ne);
      T.wtiles.push_back(w);
      plan.stats.rows_wide += w.nrows;
      ++plan.stats.wide_tiles;
    }
  }
}

// Narrow wide-row tiles (see NarrowTile): runs of NARROW_ROWS consecutive rows.
static void build_narrow(Plan& plan) {
  HostTables& T = plan.host;
  T.seg_narrow.assign(T.segs.size(), 0);
  T.ntiles.clear();
  plan.stats.rows_narrow = 0;
  if (plan.layout.order != HBC_POINT_MAJOR) return;
  const int64_t es = plan.dtype == HBC_F64 ? 8 : 4;
  if (plan.layout.inner * es >= NARROW_ROW_BYTES) return;
  for (size_t si = 0; si < T.segs.size(); ++si) {
    const DevSeg& sg = T.segs[si];
    if (sg.kind != SEG_CSR || sg.nrows == 0 || T.seg_wide[si]) continue;
    const int64_t nnz = T.csr_ptr[sg.tab + sg.nrows] - T.csr_ptr[sg.tab];
    if (nnz < WIDE_NNZ * sg.nrows) continue;
    T.seg_narrow[si] = 1;
    for (int64_t r = 0; r < sg.nrows; r += NARROW_ROWS) {
      NarrowTile t{};
      t.rot = sg.rot;
      t.has_b = sg.has_b;
      t.b_inner = sg.b_inner;
      t.nrows = (int32_t)std::min<int64_t>(NARROW_ROWS, sg.nrows - r);
      t.row_begin = sg.row_base + r;
      t.tab = sg.tab + r;
      t.brow = sg.brow + r * sg.b_inner;
      T.ntiles.push_back(t);
      plan.stats.rows_narrow += t.nrows;
    }
  }
}

// Sliding-window runs (see WinRun).  A segment qualifies when every row is a
// window (four cells c, c + dl, c + 2 dl, c + 3 dl, dl != 0).  Its rows are
// cut, in device order, into runs of at most rmax rows in which each row's
// window starts one cell further along the same line than the previous
// row's; a new run starts where that fails (at the next ghost layer of a
// strip, or where two neighbouring ghosts share a stencil).  Rows of other
// segments keep the row tiles.
static void build_windows(Plan& plan, int rmax) {
  HostTables& T = plan.host;
  T.seg_win.assign(T.segs.size(), 0);
  T.wruns.clear();
  T.win_maxr = 0;
  T.win_has_b = false;
  plan.stats.rows_window = plan.stats.window_runs = 0;
  if (!windows_possible(plan)) return;
  rmax = std::max(1, std::min(rmax, WIN_MAXR));
  for (size_t si = 0; si < T.segs.size(); ++si) {
    const DevSeg& sg = T.segs[si];
    if (!win_seg_shape(plan, sg)) continue;
    if (T.seg_wide.size() == T.segs.size() && T.seg_wide[si]) continue;
    const int32_t* c = T.ell_col.data() + sg.tab;
    auto dl_of = [&](int64_t r) { return (int64_t)c[4 * r + 1] - c[4 * r]; };
    bool ok = true;
    for (int64_t r = 0; r < sg.nrows && ok; ++r) {
      const int64_t dl = dl_of(r);
      ok = dl != 0 && dl > INT32_MIN && dl < INT32_MAX;
      for (int m = 2; m < 4 && ok; ++m) ok = (int64_t)c[4 * r + m] - c[4 * r] == m * dl;
    }
    if (!ok) continue;
    T.seg_win[si] = 1;
    int64_t r0 = 0;
    while (r0 < sg.nrows) {
      const int64_t dl = dl_of(r0);
      int64_t n = 1;
      while (r0 + n < sg.nrows && n < rmax) {
        const int64_t r = r0 + n;
        if (dl_of(r) != dl || (int64_t)c[4 * r] - c[4 * (r - 1)] != dl) break;
        ++n;
      }
      WinRun w{};
      w.src0 = c[4 * r0];
      w.dl = (int32_t)dl;
      w.nrows = (int32_t)n;
      w.nsrc = (int32_t)(n + 3);
      w.row_begin = sg.row_base + r0;
      w.tab = sg.tab + 4 * r0;
      w.brow = sg.brow + r0 * sg.b_inner;
      w.rot = sg.rot;
      w.has_b = sg.has_b;
      w.b_inner = sg.b_inner;
      T.wruns.push_back(w);
      T.win_maxr = std::max<int32_t>(T.win_maxr, (int32_t)n);
      T.win_has_b = T.win_has_b || sg.has_b;
      r0 += n;
    }
    plan.stats.rows_window += sg.nrows;
  }
  plan.stats.window_runs = (int64_t)T.wruns.size();
}

void build_tiles(Plan& plan, const hbc_tune& t) {
  if (t.block < 64 || t.block > 256 || t.block % 64) fail(HBC_EINVAL, "block must be 64, 128, 192 or 256");
  if (t.lanes_per_row < 1 || (t.lanes_per_row & (t.lanes_per_row - 1)) || t.lanes_per_row > t.block)
    fail(HBC_EINVAL, "lanes_per_row must be a power of two <= block");
  if (t.rows_per_tile < 1) fail(HBC_EINVAL, "rows_per_tile must be >= 1");
  if (t.persistent < 0) fail(HBC_EINVAL, "persistent must be >= 0");
  if (t.window_order != 0 && t.window_order != 1) fail(HBC_EINVAL, "window_order must be 0 or 1");
  std::vector<DevTile> tiles;
  for (size_t s = 0; s < plan.host.segs.size(); ++s) {
    const DevSeg& sg = plan.host.segs[s];
    for (int64_t r0 = 0; r0 < sg.nrows; r0 += t.rows_per_tile) {
      DevTile tl;
      tl.seg = (int32_t)s;
      tl.nrows = (int32_t)std::min<int64_t>(t.rows_per_tile, sg.nrows - r0);
      tl.row0 = r0;
      tiles.push_back(tl);
    }
  }
  // Workgroups are dealt to the 8 XCDs round-robin; interleave so that each
  // XCD walks a contiguous run of tiles (neighbouring rows share sources).
  const size_t n = tiles.size();
  std::vector<DevTile> out(n);
  const size_t X = 8;
  if (n >= X * 2) {
    size_t per = (n + X - 1) / X;
    size_t i = 0;
    for (size_t k = 0; k < per * X; ++k) {
      size_t x = k % X, j = k / X;
      size_t src = x * per + j;
      if (src < n) out[i++] = tiles[src];
    }
  } else {
    out = tiles;
  }
  plan.host.tiles.swap(out);
  plan.stats.tiles = (int64_t)plan.host.tiles.size();
  plan.tune = t;
  // the same cut as point-major row tiles (same XCD-aware order)
  plan.host.rtiles.clear();
  if (plan.host.seg_wide.size() != plan.host.segs.size()) build_wide(plan);
  if (plan.host.seg_narrow.size() != plan.host.segs.size()) build_narrow(plan);
  build_windows(plan, t.rows_per_tile);
  for (const DevTile& tl : plan.host.tiles) {
    const DevSeg& sg = plan.host.segs[tl.seg];
    if (plan.host.seg_wide[tl.seg] || plan.host.seg_narrow[tl.seg]) continue;  // served by the wide-row kernels
    if (plan.host.seg_win[tl.seg]) continue;                                     // served by the window kernel
    RowTile rt{};
    rt.kind = sg.kind;
    rt.rot = sg.rot;
    rt.flags = sg.flags;
    rt.width = sg.width;
    rt.row_begin = sg.row_base + tl.row0;
    rt.tab = sg.kind == SEG_ELL ? sg.tab + tl.row0 * sg.width : sg.tab + tl.row0;
    rt.brow = sg.brow + tl.row0 * sg.b_inner;
    rt.w = sg.w;
    rt.nrows = tl.nrows;
    rt.has_b = sg.has_b;
    rt.b_inner = sg.b_inner;
    plan.host.rtiles.push_back(rt);
  }
}

// Tiles of the LDS-staged adjoint: consecutive sources, greedily, while the
// distinct ghost rows of the tile fit the LDS rows and the tile stays short
// enough to leave many workgroups in flight.
static void build_adj_lds(Plan& plan) {
  const CscHost& C = plan.host.csc;
  AdjLdsHost& A = plan.host.adj_lds;
  A = AdjLdsHost{};
  if (plan.layout.order != HBC_POINT_MAJOR) return;
  const int64_t row_bytes = plan.layout.inner * (plan.dtype == HBC_F64 ? 8 : 4);
  const int64_t brows = std::min<int64_t>(ADJ_LDS_ROWS, ADJ_LDS_BYTES / std::max<int64_t>(1, row_bytes));
  const int64_t nsrc = (int64_t)C.src_cell.size();
  int64_t maxc = 0;
  for (int64_t k = 0; k < nsrc; ++k) maxc = std::max<int64_t>(maxc, C.cnt[k]);
  if (maxc > C.aw || maxc > brows || brows < 1) return;  // the CSR-walking kernel serves such plans
  A.brows = (int32_t)brows;
  // sources per tile: at most 256 (about 4 per row group of the adjoint's
  // launch shape); the ghost-row limit is the one that binds in practice
  const int64_t smax = 256;
  A.slot.assign((size_t)nsrc * C.aw, 0);
  std::unordered_map<int64_t, int32_t> local;
  std::unordered_map<int64_t, int32_t> readers;  // ghost -> reader tiles
  int64_t k = 0;
  while (k < nsrc) {
    AdjLdsTile t{(int32_t)k, 0, (int32_t)A.u_cell.size(), 0};
    local.clear();
    while (k < nsrc && t.nsrc < smax) {
      int add = 0;
      for (int32_t m = 0; m < C.cnt[k]; ++m)
        if (!local.count(C.fghost[k * C.aw + m])) ++add;
      // (a ghost repeated within one source is counted twice: conservative)
      if (t.nu + add > brows) break;
      for (int32_t m = 0; m < C.cnt[k]; ++m) {
        const int64_t g = C.fghost[k * C.aw + m];
        auto it = local.find(g);
        int32_t sl;
        if (it == local.end()) {
          sl = t.nu++;
          local.emplace(g, sl);
          A.u_cell.push_back((int32_t)g);
          ++readers[g];
        } else {
          sl = it->second;
        }
        A.slot[k * C.aw + m] = (uint16_t)sl;
      }
      ++t.nsrc;
      ++k;
    }
    if (t.nsrc == 0) return;  // cannot happen: every source fits an empty tile
    A.tiles.push_back(t);
  }
  std::unordered_map<int64_t, int32_t> ctr_of;
  A.u_ctr.assign(A.u_cell.size(), -1);
  for (size_t u = 0; u < A.u_cell.size(); ++u) {
    const int64_t g = A.u_cell[u];
    const int32_t n = readers[g];
    if (n < 2) continue;
    auto it = ctr_of.find(g);
    if (it == ctr_of.end()) {
      it = ctr_of.emplace(g, (int32_t)A.ctr_init.size()).first;
      A.ctr_init.push_back(n);
    }
    A.u_ctr[u] = it->second;
  }
  for (int32_t r : plan.host.row_dst)
    if (!readers.count(r)) A.zero_rows.push_back(r);
  A.ok = true;
}

void build_csc(Plan& plan) {
  const HostTables& T = plan.host;
  struct E {
    int64_t src, ghost;
    double w;
    int32_t rot;
  };
  std::vector<E> ents;
  ents.reserve((size_t)plan.stats.nnz);
  for (const DevSeg& s : T.segs) {
    const int irot = rot_inverse(s.rot);
    int64_t c[SEG_MAXD];
    for (int64_t r = 0; r < s.nrows; ++r) {
      int64_t q = r;
      for (int d = s.nd - 1; d >= 0; --d) {
        c[d] = q % s.ext[d];
        q /= s.ext[d];
      }
      int64_t dst = s.dst_base, src = s.src_base;
      for (int d = 0; d < s.nd; ++d) {
        dst += c[d] * s.dst_stride[d];
        src += c[d] * s.src_stride[d];
      }
      if (s.kind == SEG_MAP) {
        ents.push_back(E{src, dst, s.w, irot});
      } else if (s.kind == SEG_ELL) {
        for (int m = 0; m < s.width; ++m) {
          int32_t col = T.ell_col[s.tab + r * s.width + m];
          if (col >= 0) ents.push_back(E{col, dst, T.ell_val[s.tab + r * s.width + m], irot});
        }
      } else if (s.kind == SEG_CSR) {
        for (int64_t k = T.csr_ptr[s.tab + r]; k < T.csr_ptr[s.tab + r + 1]; ++k)
          ents.push_back(E{T.csr_col[k], dst, T.csr_val[k], irot});
      }
    }
  }
  std::sort(ents.begin(), ents.end(), [](const E& a, const E& b) {
    return a.src != b.src ? a.src < b.src : a.ghost < b.ghost;
  });
  CscHost& C = plan.host.csc;
  C = CscHost{};
  for (size_t k = 0; k < ents.size(); ++k) {
    if (k == 0 || ents[k].src != ents[k - 1].src) {
      C.src_cell.push_back(ents[k].src);
      C.ptr.push_back((int64_t)k);
    }
    C.ghost.push_back(ents[k].ghost);
    C.w.push_back(ents[k].w);
    C.rot.push_back(ents[k].rot);
  }
  C.ptr.push_back((int64_t)ents.size());
  const int64_t nsrc = (int64_t)C.src_cell.size();
  int64_t maxc = 0;
  for (int64_t k = 0; k < nsrc; ++k) maxc = std::max(maxc, C.ptr[k + 1] - C.ptr[k]);
  C.aw = (int32_t)std::max<int64_t>(1, std::min<int64_t>(maxc, ADJ_MAXW));
  C.cnt.assign(nsrc, 0);
  C.fghost.assign(nsrc * C.aw, 0);
  C.fw.assign(nsrc * C.aw, 0.0);
  C.frot.assign(nsrc * C.aw, 0);
  for (int64_t k = 0; k < nsrc; ++k) {
    const int64_t n = C.ptr[k + 1] - C.ptr[k];
    C.cnt[k] = (int32_t)n;
    for (int64_t m = 0; m < std::min<int64_t>(n, C.aw); ++m) {
      const int64_t e = C.ptr[k] + m;
      C.fghost[k * C.aw + m] = (int32_t)C.ghost[e];
      C.fw[k * C.aw + m] = C.w[e];
      C.frot[k * C.aw + m] = (int8_t)C.rot[e];
    }
  }
  build_adj_lds(plan);
  // adjoint tiles: sources grouped so that a tile holds about as many inner
  // values as a forward tile
  plan.host.adj_tiles.clear();
  const int64_t ns = (int64_t)C.src_cell.size();
  int64_t per = std::max<int64_t>(plan.tune.block / plan.tune.lanes_per_row, ns / 2048);
  per = std::min<int64_t>(per, 16384);
  for (int64_t s = 0; s < ns; s += per)
    plan.host.adj_tiles.push_back(AdjTile{(int32_t)s, (int32_t)std::min<int64_t>(per, ns - s)});
}

// ---- 27-point consumer: which block each one-cell ghost region copies from ------------------
// Plays the role of the dependence analysis of Sec. IV-C for this consumer:
// every ghost the stencil reads is traced to the BC row that writes it, and
// the fused kernel is allowed only when each of a block's 26 ghost regions is
// one translated copy of a neighbouring block (or zero, or left uncovered).
void compute_stencil_info(Plan& p) {
  p.st_ok = p.st_fused = false;
  const Grid& g = p.grid;
  auto no = [&](const char* why) { p.st_reason = p.st_fused_reason = why; };
  if (g.nd != 4) return no("the 27-point consumer needs a Cartesian block grid (block, z, y, x)");
  if (p.layout.inner != 1) return no("the 27-point consumer needs inner == 1");
  const Block& B0 = g.blocks[0];
  int64_t n[3];
  for (int d = 0; d < 3; ++d) n[d] = B0.data.extent(d + 1);
  for (const Block& B : g.blocks) {
    if (B.full.extent(0) != 1) return no("blocks must have extent 1 along coordinate 0");
    for (int d = 0; d < 3; ++d)
      if (B.data.extent(d + 1) != n[d] || B.data.lo[d + 1] - B.full.lo[d + 1] != 1 ||
          B.full.hi[d + 1] - B.data.hi[d + 1] != 1)
        return no("the 27-point consumer needs equal blocks with a one-cell halo");
  }
  const int nb = (int)g.blocks.size();
  for (int d = 0; d < 3; ++d) p.st_n[d] = n[d];
  p.st_nblocks = nb;
  p.st_ok = true;  // the unfused form reads the ghosts x holds
  auto no_fused = [&](const char* why) { p.st_fused_reason = why; };
  if (p.stats.rows_data > 0) return no_fused("the fused 27-point consumer does not take data rows");
  std::vector<int64_t> info((size_t)nb * 27, -3);
  for (int b = 0; b < nb; ++b) info[(size_t)b * 27 + 13] = b;
  std::vector<int64_t> firsts(nb);
  for (int b = 0; b < nb; ++b) firsts[b] = g.blocks[b].first_cell;
  const HostTables& T = p.host;
  std::vector<int64_t> rows_in((size_t)nb * 27, 0);  // covered rows per block and direction
  bool ok = true;
  for (size_t si = 0; si < T.segs.size() && ok; ++si) {
    const DevSeg& sg = T.segs[si];
    const Box& bx = T.seg_box[si];
    const int b = g.owner(bx.lo);
    const Block& B = g.blocks[b];
    for_box_order(bx, T.seg_order[si], [&](const int64_t* c, int64_t r) {
      if (!ok) return;
      int64_t pl[3];
      int dd[3];
      for (int d = 0; d < 3; ++d) {
        pl[d] = c[d + 1] - B.data.lo[d + 1];
        dd[d] = pl[d] < 0 ? -1 : (pl[d] >= n[d] ? 1 : 0);
      }
      const int di = (dd[0] + 1) * 9 + (dd[1] + 1) * 3 + (dd[2] + 1);
      int64_t v;
      if (sg.kind == SEG_ZERO && !sg.has_b) {
        v = -1;
      } else if (sg.kind == SEG_MAP && sg.w == 1.0 && sg.rot == 0 && !sg.has_b) {
        const int64_t src = T.row_src[sg.row_base + r];
        const int ob = (int)(std::upper_bound(firsts.begin(), firsts.end(), src) - firsts.begin()) - 1;
        const Block& O = g.blocks[ob];
        int64_t off = src - O.first_cell;
        bool match = true;
        for (int d = 0; d < 4; ++d) {
          const int64_t cd = O.full.lo[d] + off / O.stride[d];
          off %= O.stride[d];
          if (d > 0 && cd - O.data.lo[d] != pl[d - 1] - dd[d - 1] * n[d - 1]) match = false;
        }
        if (!match) {
          ok = false;
          no_fused("a halo copy is not a translation by one block");
          return;
        }
        v = ob;
      } else {
        ok = false;
        no_fused("the fused consumer supports copy and zero rows only");
        return;
      }
      ++rows_in[(size_t)b * 27 + di];
      int64_t& slot = info[(size_t)b * 27 + di];
      if (slot == -3) {
        slot = v;
      } else if (slot != v) {
        ok = false;
        no_fused("one ghost region mixes BC kinds or source blocks");
      }
    });
  }
  if (!ok) return;
  // the fused form reads a whole region through the BC: every cell of a
  // covered region must have its row
  for (int b = 0; b < nb; ++b)
    for (int di = 0; di < 27; ++di) {
      if (di == 13 || info[(size_t)b * 27 + di] == -3) continue;
      const int dd[3] = {di / 9 - 1, di / 3 % 3 - 1, di % 3 - 1};
      int64_t cells = 1;
      for (int d = 0; d < 3; ++d) cells *= dd[d] == 0 ? n[d] : 1;
      if (rows_in[(size_t)b * 27 + di] != cells) return no_fused("a ghost region of the 27-point consumer is only partly covered");
    }
  for (int64_t& v : info)
    if (v == -3) v = -2;
  p.st_info.swap(info);
  p.st_fused = true;
}

// ---- host evaluation of compiled rows (tests without a GPU) --------------------------------
int plan_row(const Plan& plan, int64_t cell, int64_t l, int cap, int64_t* cols, double* vals, int32_t* nnz,
             double* b, int32_t* kind, int32_t* rot) {
  const HostTables& T = plan.host;
  const Grid& g = plan.grid;
  *nnz = 0;
  *b = 0.0;
  *kind = -1;
  *rot = 0;
  // global coordinates of the cell
  int blk = -1;
  for (size_t k = 0; k < g.blocks.size(); ++k)
    if (cell >= g.blocks[k].first_cell && cell < g.blocks[k].first_cell + g.blocks[k].cells) blk = (int)k;
  if (blk < 0) return HBC_OK;
  for (size_t k = 0; k < T.dr_cell.size(); ++k) {
    if (T.dr_cell[k] != cell) continue;  // a data row (kind SEG_DATA_ROW)
    *kind = SEG_DATA_ROW;
    int n = 0;
    for (int64_t e = T.dr_ptr[k]; e < T.dr_ptr[k + 1]; ++e, ++n)
      if (n < cap) {
        cols[n] = T.dr_col[e];
        vals[n] = T.dr_val[e];
      }
    *nnz = n;
    return HBC_OK;
  }
  int64_t c[HBC_MAX_DIM];
  int64_t off = cell - g.blocks[blk].first_cell;
  for (int d = 0; d < g.nd; ++d) {
    c[d] = g.blocks[blk].full.lo[d] + off / g.blocks[blk].stride[d];
    off %= g.blocks[blk].stride[d];
  }
  for (size_t si = 0; si < T.segs.size(); ++si) {
    if (!T.seg_box[si].contains(c)) continue;
    const DevSeg& s = T.segs[si];
    const Box& bx = T.seg_box[si];
    int64_t r = 0;
    for (int d : T.seg_order[si]) r = r * bx.extent(d) + (c[d] - bx.lo[d]);
    *kind = s.kind;
    *rot = s.rot;
    if (s.kind == SEG_MAP) {
      // row r's coordinates in the device order -> source cell
      int64_t q = r, src = s.src_base;
      for (int d = s.nd - 1; d >= 0; --d) {
        src += (q % s.ext[d]) * s.src_stride[d];
        q /= s.ext[d];
      }
      if (cap > 0) {
        cols[0] = src;
        vals[0] = s.w;
      }
      *nnz = 1;
    } else if (s.kind == SEG_ELL) {
      int n = 0;
      for (int m = 0; m < s.width; ++m) {
        int32_t col = T.ell_col[s.tab + r * s.width + m];
        if (col < 0) continue;
        if (n < cap) {
          cols[n] = col;
          vals[n] = T.ell_val[s.tab + r * s.width + m];
        }
        ++n;
      }
      *nnz = n;
    } else if (s.kind == SEG_CSR) {
      int n = 0;
      for (int64_t k = T.csr_ptr[s.tab + r]; k < T.csr_ptr[s.tab + r + 1]; ++k, ++n)
        if (n < cap) {
          cols[n] = T.csr_col[k];
          vals[n] = T.csr_val[k];
        }
      *nnz = n;
    }
    if (s.has_b) *b = T.bval[s.brow + r * s.b_inner + (s.b_inner == 1 ? 0 : l)];
    return HBC_OK;
  }
  return HBC_OK;
}

}  // namespace hbc
