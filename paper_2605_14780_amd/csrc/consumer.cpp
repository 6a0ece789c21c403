// Consumer of the BC's ghosts (Sec. IV-C: the boundary writes exist to feed
// the inner computation that follows; the two share one representation and
// are optimised together).  The consumer is a stencil given by offsets and
// weights, y[c] = sum_o w_o x'[c + o] over every data cell c, x' the field
// after the apply.  This file compiles it against a plan: cell deltas of the
// offsets per block, structured tiles for the cells whose reads are all data
// cells, and, for the others, the stencil composed with the compiled BC rows
// of the ghosts it reaches.
#include <algorithm>
#include <cstring>
#include <unordered_map>

#include "hbc_internal.hpp"

namespace hbc {

namespace {

// Row-major runs along the last dimension of box bx (inside block b), cut into
// tiles of at most tile_cells cells; y0 is the output row of the box's first
// cell in the block's data box, ybase the block's first output row.
void box_tiles(const Grid& g, int b, const Box& bx, const Box& data, int64_t ybase, int tile_cells,
               std::vector<CTile>& out) {
  if (bx.empty()) return;
  const Block& B = g.blocks[b];
  const int nd = g.nd;
  int64_t c[HBC_MAX_DIM];
  for (int d = 0; d < nd; ++d) c[d] = bx.lo[d];
  const int64_t nlast = bx.extent(nd - 1);
  while (true) {
    int64_t cell = B.first_cell, yrow = 0;
    for (int d = 0; d < nd; ++d) {
      cell += (c[d] - B.full.lo[d]) * B.stride[d];
      yrow = yrow * data.extent(d) + (c[d] - data.lo[d]);
    }
    for (int64_t k = 0; k < nlast; k += tile_cells) {
      CTile t;
      t.cell0 = (int32_t)(cell + k);
      t.y0 = (int32_t)(ybase + yrow + k);
      t.n = (int32_t)std::min<int64_t>(tile_cells, nlast - k);
      t.blk = b;
      out.push_back(t);
    }
    int d = nd - 2;  // advance over all but the last dimension
    for (; d >= 0; --d) {
      if (++c[d] < bx.hi[d]) break;
      c[d] = bx.lo[d];
    }
    if (d < 0) break;
  }
}

// Lines of the offsets: offsets equal in all but the last dimension.  When
// they lie on at most CONS_MAXLINES lines, each within +-1 along the last
// dimension and without repeats, the structured walk keeps a ring of each
// line's last three points (one new load per line and cell), and the
// offsets are reordered line by line (lines in order of first appearance,
// each in ascending last coordinate): the order of every sum, in both forms.
// Returns the offsets per line (empty: the general walk).
std::vector<int> find_lines(int nd, ConsumerHost& C) {
  const int noff = C.noff;
  std::vector<std::vector<int>> lines;
  for (int o = 0; o < noff; ++o) {
    const int64_t p = C.off[(size_t)o * nd + nd - 1];
    if (p < -1 || p > 1) return {};
    size_t l = 0;
    for (; l < lines.size(); ++l) {
      const int f = lines[l][0];
      bool same = true;
      for (int d = 0; d + 1 < nd; ++d) same = same && C.off[(size_t)f * nd + d] == C.off[(size_t)o * nd + d];
      if (same) break;
    }
    if (l == lines.size()) {
      if (lines.size() == (size_t)CONS_MAXLINES) return {};
      lines.emplace_back();
    }
    for (int q : lines[l])
      if (C.off[(size_t)q * nd + nd - 1] == p) return {};  // a repeated offset
    lines[l].push_back(o);
  }
  std::vector<int64_t> off;
  std::vector<double> w;
  std::vector<int> len;
  C.line_w.assign(lines.size() * 3, 0.0);
  C.line_mask = 0;
  for (size_t l = 0; l < lines.size(); ++l) {
    std::vector<int>& L = lines[l];
    std::sort(L.begin(), L.end(), [&](int a, int b) { return C.off[(size_t)a * nd + nd - 1] < C.off[(size_t)b * nd + nd - 1]; });
    const int64_t pmax = C.off[(size_t)L.back() * nd + nd - 1];
    for (int o : L) {
      off.insert(off.end(), C.off.begin() + (size_t)o * nd, C.off.begin() + (size_t)(o + 1) * nd);
      w.push_back(C.w[o]);
      const int s = (int)(C.off[(size_t)o * nd + nd - 1] - pmax + 2);
      C.line_w[l * 3 + s] = C.w[o];
      C.line_mask |= 1 << (3 * l + s);
    }
    len.push_back((int)L.size());
  }
  C.off.swap(off);
  C.w.swap(w);
  C.nlines = (int)lines.size();
  return len;
}

}  // namespace

void compile_consumer(const Plan& plan, int noff, const int64_t* offsets, const double* weights, ConsumerHost& C) {
  const Grid& g = plan.grid;
  const int nd = g.nd;
  if (noff < 1 || noff > CONS_MAXOFF) fail(HBC_EINVAL, "the consumer needs 1 to 64 offsets");
  if (plan.layout.order != HBC_POINT_MAJOR) fail(HBC_EUNSUPPORTED, "the consumer needs the point-major layout");
  if (plan.stats.rows_data > 0) fail(HBC_EUNSUPPORTED, "no consumer for plans with data rows");
  C = ConsumerHost{};
  C.noff = noff;
  C.off.resize((size_t)noff * nd);
  for (int o = 0; o < noff; ++o)
    for (int d = 0; d < nd; ++d) {
      const int64_t v = offsets[(size_t)o * nd + d];
      if (v % g.step[d] != 0) fail(HBC_EINVAL, "consumer offsets must be multiples of the grid's step");
      C.off[(size_t)o * nd + d] = v / g.step[d];
    }
  C.w.assign(weights, weights + noff);
  const std::vector<int> line_len = find_lines(nd, C);
  // every read of every data cell stays inside its block's full box
  C.delta.resize(g.blocks.size() * (size_t)noff);
  for (size_t b = 0; b < g.blocks.size(); ++b) {
    const Block& B = g.blocks[b];
    for (int o = 0; o < noff; ++o) {
      int64_t dl = 0;
      for (int d = 0; d < nd; ++d) {
        const int64_t v = C.off[(size_t)o * nd + d];
        if (B.data.lo[d] + v < B.full.lo[d] || B.data.hi[d] + v > B.full.hi[d])
          fail(HBC_EINVAL, "a consumer offset reads outside block " + std::to_string(b) + "'s full region");
        dl += v * B.stride[d];
      }
      C.delta[b * noff + o] = (int32_t)dl;
    }
  }
  // each line's last point: its last offset (the lines' offsets are consecutive)
  C.line_delta.resize(g.blocks.size() * (size_t)C.nlines);
  for (size_t b = 0, o = 0; b < g.blocks.size(); ++b, o = 0)
    for (int l = 0; l < C.nlines; ++l) {
      o += (size_t)line_len[l];
      C.line_delta[b * C.nlines + l] = C.delta[b * noff + o - 1];
    }
  const int lpr = std::max(1, plan.tune.lanes_per_row), groups = std::max(1, 256 / lpr);
  C.tile_cells = groups * CONS_CELLS;
  C.tile_rows = groups * CONS_BROWS;
  // covered ghost rows: cell -> row of the plan's device order
  const HostTables& T = plan.host;
  std::unordered_map<int32_t, int64_t> row_of;
  row_of.reserve(T.row_dst.size() * 2);
  for (size_t k = 0; k < T.row_dst.size(); ++k) row_of.emplace(T.row_dst[k], (int64_t)k);
  std::vector<int64_t> seg_start(T.segs.size());
  for (size_t s = 0; s < T.segs.size(); ++s) seg_start[s] = T.segs[s].row_base;
  const int64_t I = plan.layout.inner;
  int64_t ybase = 0;
  std::vector<double> brow(I);
  for (size_t b = 0; b < g.blocks.size(); ++b) {
    const Block& B = g.blocks[b];
    const Box& D = B.data;
    box_tiles(g, (int)b, D, D, ybase, C.tile_cells, C.tiles_all);
    // interior: D shrunk by the offsets' reach in each direction
    Box in = D;
    for (int d = 0; d < nd; ++d)
      for (int o = 0; o < noff; ++o) {
        const int64_t v = C.off[(size_t)o * nd + d];
        in.lo[d] = std::max(in.lo[d], D.lo[d] - std::min<int64_t>(v, 0));
        in.hi[d] = std::min(in.hi[d], D.hi[d] - std::max<int64_t>(v, 0));
      }
    bool has_in = true;
    for (int d = 0; d < nd; ++d) has_in = has_in && in.lo[d] < in.hi[d];
    if (has_in) box_tiles(g, (int)b, in, D, ybase, C.tile_cells, C.tiles_int);
    // boundary rows: the data cells outside the interior box, in output order
    int64_t c[HBC_MAX_DIM];
    for (int d = 0; d < nd; ++d) c[d] = D.lo[d];
    int64_t yrow = 0;
    while (true) {
      if (!(has_in && in.contains(c))) {
        const int64_t cell = g.cell((int)b, c);
        std::fill(brow.begin(), brow.end(), 0.0);
        bool with_b = false;
        C.brow_y.push_back((int32_t)(ybase + yrow));
        C.bptr.push_back((int32_t)C.bcol.size());
        for (int o = 0; o < noff; ++o) {
          const double wo = C.w[o];
          int64_t n[HBC_MAX_DIM];
          for (int d = 0; d < nd; ++d) n[d] = c[d] + C.off[(size_t)o * nd + d];
          const int64_t nc = cell + C.delta[b * noff + o];
          auto it = D.contains(n) ? row_of.end() : row_of.find((int32_t)nc);
          if (D.contains(n) || it == row_of.end()) {
            // a data cell, or a ghost no sub-matrix covers (read as stored)
            C.bcol.push_back((int32_t)nc);
            C.bw.push_back(wo);
            C.brot.push_back(0);
            continue;
          }
          const int64_t k = it->second;
          const size_t si = (size_t)(std::upper_bound(seg_start.begin(), seg_start.end(), k) - seg_start.begin()) - 1;
          const DevSeg& s = T.segs[si];
          const int64_t r = k - s.row_base;
          auto add = [&](int64_t col, double v) {
            C.bcol.push_back((int32_t)col);
            C.bw.push_back(wo * v);
            C.brot.push_back((int8_t)s.rot);
          };
          if (s.kind == SEG_MAP) {
            add(T.row_src[k], s.w);
          } else if (s.kind == SEG_ELL) {
            for (int m = 0; m < s.width; ++m) {
              const int32_t col = T.ell_col[s.tab + r * s.width + m];
              if (col >= 0) add(col, T.ell_val[s.tab + r * s.width + m]);
            }
          } else if (s.kind == SEG_CSR) {
            for (int64_t e = T.csr_ptr[s.tab + r]; e < T.csr_ptr[s.tab + r + 1]; ++e) add(T.csr_col[e], T.csr_val[e]);
          }
          if (s.has_b) {
            with_b = true;
            for (int64_t l = 0; l < I; ++l) brow[l] += wo * T.bval[s.brow + r * s.b_inner + (s.b_inner == 1 ? 0 : l)];
          }
        }
        if (with_b) {
          C.bconst_row.push_back((int32_t)(C.bconst.size() / I));
          C.bconst.insert(C.bconst.end(), brow.begin(), brow.end());
        } else {
          C.bconst_row.push_back(-1);
        }
      }
      ++yrow;
      int d = nd - 1;
      for (; d >= 0; --d) {
        if (++c[d] < D.hi[d]) break;
        c[d] = D.lo[d];
      }
      if (d < 0) break;
    }
    ybase += D.count();
  }
  C.bptr.push_back((int32_t)C.bcol.size());
  C.ndata = ybase;
}

}  // namespace hbc
