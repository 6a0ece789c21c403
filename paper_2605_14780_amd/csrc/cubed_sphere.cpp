// Cubed-sphere BC programs from integer face frames.
//
// Sec. II-B: a ghost of one panel is seen from the neighbouring panel and
// interpolated there; Alg. 1 gives a copy whose axes are rotated between
// blocks.  The connectivity of the six faces, the mirrored grid line and the
// direction of the tangential index are derived here exactly, from integer
// frame vectors (centre c, tangents e1, e2 with c x e1 = e2), so no floating
// point decides an index.
#include <algorithm>
#include <cmath>
#include <map>
#include <cstring>
#include <numeric>
#include <vector>

#include "hbc_internal.hpp"

namespace hbc {
namespace {

struct V3 {
  int x, y, z;
};
int dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
V3 neg(V3 a) { return V3{-a.x, -a.y, -a.z}; }
V3 add(V3 a, V3 b) { return V3{a.x + b.x, a.y + b.y, a.z + b.z}; }
V3 scale(V3 a, int s) { return V3{a.x * s, a.y * s, a.z * s}; }
bool eq(V3 a, V3 b) { return a.x == b.x && a.y == b.y && a.z == b.z; }

// face frames: f0 (+x,+y,+z), f1 (+y,-x,+z), f2 (-x,-y,+z), f3 (-y,+x,+z),
// f4 (+z,+y,-x), f5 (-z,+y,+x)
const V3 FR[6][3] = {
    {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}},  {{0, 1, 0}, {-1, 0, 0}, {0, 0, 1}}, {{-1, 0, 0}, {0, -1, 0}, {0, 0, 1}},
    {{0, -1, 0}, {1, 0, 0}, {0, 0, 1}}, {{0, 0, 1}, {0, 1, 0}, {-1, 0, 0}}, {{0, 0, -1}, {0, 1, 0}, {1, 0, 0}},
};

enum { LEFT = 0, RIGHT = 1, BOTTOM = 2, TOP = 3 };

V3 outward(int f, int side) {
  switch (side) {
    case LEFT: return neg(FR[f][1]);
    case RIGHT: return FR[f][1];
    case BOTTOM: return neg(FR[f][2]);
    default: return FR[f][2];
  }
}

struct SideLink {
  int g;       // neighbour face
  int gside;   // side of g facing f
  bool rev;    // tangential index runs backwards on g
  int rot[4];  // 2x2 component rotation (ghost components from neighbour components)
};

// tangent of the alpha (axis 0) or beta (axis 1) lines of face F at the point
// P = c + a e1 + b e2, scaled to integers: e |P|^2 - P (P.e)
V3 tangent(int F, int axis, int a, int b) {
  V3 P = add(FR[F][0], add(scale(FR[F][1], a), scale(FR[F][2], b)));
  int n2 = 1 + a * a + b * b;
  V3 e = FR[F][1 + axis];
  return add(scale(e, n2), scale(P, -(axis == 0 ? a : b)));
}

SideLink link(int f, int side) {
  SideLink L{};
  V3 n = outward(f, side);
  L.g = -1;
  for (int g = 0; g < 6; ++g)
    if (eq(FR[g][0], n)) L.g = g;
  const int g = L.g;
  V3 cf = FR[f][0];
  if (eq(FR[g][1], neg(cf))) L.gside = LEFT;
  else if (eq(FR[g][1], cf)) L.gside = RIGHT;
  else if (eq(FR[g][2], neg(cf))) L.gside = BOTTOM;
  else L.gside = TOP;
  V3 tf = (side == LEFT || side == RIGHT) ? FR[f][2] : FR[f][1];
  V3 tg = (L.gside == LEFT || L.gside == RIGHT) ? FR[g][2] : FR[g][1];
  L.rev = dot(tf, tg) < 0;
  // component rotation at the midpoint of the shared edge
  int af = side == LEFT ? -1 : side == RIGHT ? 1 : 0;
  int bf = side == BOTTOM ? -1 : side == TOP ? 1 : 0;
  V3 Q = add(cf, n);
  int ag = dot(Q, FR[g][1]), bg = dot(Q, FR[g][2]);
  for (int p = 0; p < 2; ++p)
    for (int q = 0; q < 2; ++q) {
      int d = dot(tangent(f, p, af, bf), tangent(g, q, ag, bg));
      L.rot[p * 2 + q] = d > 0 ? 1 : d < 0 ? -1 : 0;
    }
  return L;
}

}  // namespace

void cs_add_program(Program& p, int64_t N, int64_t h, int mode, int vector, const int32_t* base, const double* w) {
  const Grid& g = p.grid;
  if (N < 4 || h < 1 || 2 * h > N)
    fail(HBC_EINVAL, "cubed sphere needs N >= 4 and 1 <= h <= N/2 (deeper ghost layers leave the face's gnomonic chart)");
  if (g.nd != 3 || g.blocks.size() != 6 || g.blocks[0].data.extent(1) != N ||
      g.blocks[0].full.lo[1] != -h || g.blocks[0].full.hi[1] != N + h)
    fail(HBC_EINVAL, "program grid is not the cubed-sphere grid of this N and h");
  if (mode != HBC_CS_SYNC && mode != HBC_CS_LAGRANGE) fail(HBC_EINVAL, "unknown cubed-sphere mode");
  if (mode == HBC_CS_LAGRANGE && (!base || !w)) fail(HBC_EINVAL, "Lagrange mode needs base and weights");
  const int64_t W = N + 2 * h;  // full extent per face dimension
  auto lin = [&](int64_t f, int64_t j, int64_t i) { return (f * W + (j + h)) * W + (i + h); };

  for (int f = 0; f < 6; ++f) {
    for (int side = 0; side < 4; ++side) {
      SideLink L = link(f, side);
      Sub s;
      s.rows.nd = 3;
      s.rows.lo[0] = f;
      s.rows.hi[0] = f + 1;
      // rows: (j, i); layer k and tangential t as affine forms in (j, i)
      if (side == LEFT) { s.rows.lo[1] = 0; s.rows.hi[1] = N; s.rows.lo[2] = -h; s.rows.hi[2] = 0; }
      if (side == RIGHT) { s.rows.lo[1] = 0; s.rows.hi[1] = N; s.rows.lo[2] = N; s.rows.hi[2] = N + h; }
      if (side == BOTTOM) { s.rows.lo[1] = -h; s.rows.hi[1] = 0; s.rows.lo[2] = 0; s.rows.hi[2] = N; }
      if (side == TOP) { s.rows.lo[1] = N; s.rows.hi[1] = N + h; s.rows.lo[2] = 0; s.rows.hi[2] = N; }
      s.rot = vector ? rot_code(L.rot) : 0;
      if (s.rot < 0) fail(HBC_EINVAL, "internal: face rotation is not a signed permutation");
      // k = kj*j + ki*i + k0 ; t = tj*j + ti*i + t0
      int64_t kj = 0, ki = 0, k0 = 0, tj = 0, ti = 0, t0 = 0;
      if (side == LEFT) { ki = -1; k0 = -1; tj = 1; }
      if (side == RIGHT) { ki = 1; k0 = -N; tj = 1; }
      if (side == BOTTOM) { kj = -1; k0 = -1; ti = 1; }
      if (side == TOP) { kj = 1; k0 = -N; ti = 1; }
      // line index on g: k (g's left/bottom side) or N-1-k (right/top)
      const bool near0 = L.gside == LEFT || L.gside == BOTTOM;
      const int64_t Ls = near0 ? 1 : -1, L0 = near0 ? 0 : N - 1;
      const int64_t Ts = L.rev ? -1 : 1, T0 = L.rev ? N - 1 : 0;
      const bool g_lr = L.gside == LEFT || L.gside == RIGHT;  // line is i = L (nodes vary in j)
      if (mode == HBC_CS_SYNC) {
        s.kind = SUB_MAP;
        s.w = 1.0;
        std::memset(s.M, 0, sizeof(s.M));
        std::memset(s.off, 0, sizeof(s.off));
        s.off[0] = L.g;
        // Lg = Ls*k + L0 ; tg = Ts*t + T0
        int64_t Lj = Ls * kj, Li = Ls * ki, Lc = Ls * k0 + L0;
        int64_t Tj = Ts * tj, Ti = Ts * ti, Tc = Ts * t0 + T0;
        if (g_lr) {  // (j_g, i_g) = (tg, Lg)
          s.M[1 * 3 + 1] = Tj; s.M[1 * 3 + 2] = Ti; s.off[1] = Tc;
          s.M[2 * 3 + 1] = Lj; s.M[2 * 3 + 2] = Li; s.off[2] = Lc;
        } else {  // (j_g, i_g) = (Lg, tg)
          s.M[1 * 3 + 1] = Lj; s.M[1 * 3 + 2] = Li; s.off[1] = Lc;
          s.M[2 * 3 + 1] = Tj; s.M[2 * 3 + 2] = Ti; s.off[2] = Tc;
        }
      } else {
        s.kind = SUB_ELL;
        s.width = 4;
        const int64_t nrow = s.rows.count();
        s.cols.resize((size_t)nrow * 4);
        s.vals.resize((size_t)nrow * 4);
        int64_t r = 0;
        for (int64_t j = s.rows.lo[1]; j < s.rows.hi[1]; ++j)
          for (int64_t i = s.rows.lo[2]; i < s.rows.hi[2]; ++i, ++r) {
            int64_t k = kj * j + ki * i + k0, t = tj * j + ti * i + t0;
            int64_t Lg = Ls * k + L0;
            int32_t b0 = base[k * N + t];
            if (b0 < 0 || b0 > N - 4) fail(HBC_EINVAL, "Lagrange base out of range");
            for (int m = 0; m < 4; ++m) {
              int64_t tg = Ts * (b0 + m) + T0;
              int64_t jg = g_lr ? tg : Lg, ig = g_lr ? Lg : tg;
              s.cols[r * 4 + m] = lin(L.g, jg, ig);
              s.vals[r * 4 + m] = w[(k * N + t) * 4 + m];
            }
          }
      }
      p.subs.push_back(std::move(s));
    }
    // corners: zero rows (h x h each)
    const int64_t lo[2] = {-h, N}, hi[2] = {0, N + h};
    for (int a = 0; a < 2; ++a)
      for (int c = 0; c < 2; ++c) {
        Sub z;
        z.kind = SUB_ZERO;
        z.rows.nd = 3;
        z.rows.lo[0] = f; z.rows.hi[0] = f + 1;
        z.rows.lo[1] = lo[a]; z.rows.hi[1] = hi[a];
        z.rows.lo[2] = lo[c]; z.rows.hi[2] = hi[c];
        p.subs.push_back(z);
      }
  }
}

void cart_add_halo(Program& p, const int32_t* nb, const int64_t* n, int64_t h, int32_t periodic) {
  const Grid& g = p.grid;
  if (h < 1) fail(HBC_EINVAL, "halo must be >= 1");
  for (int d = 0; d < 3; ++d) {
    if (nb[d] < 1 || n[d] < 1) fail(HBC_EINVAL, "block counts and sizes must be >= 1");
    if (h > n[d]) fail(HBC_EINVAL, "halo wider than a block");
  }
  const int64_t nblk = (int64_t)nb[0] * nb[1] * nb[2];
  if (g.nd != 4 || (int64_t)g.blocks.size() != nblk) fail(HBC_EINVAL, "program grid is not this Cartesian grid");
  for (int bz = 0; bz < nb[0]; ++bz)
    for (int by = 0; by < nb[1]; ++by)
      for (int bx = 0; bx < nb[2]; ++bx) {
        const int bc[3] = {bz, by, bx};
        const int64_t b = ((int64_t)bz * nb[1] + by) * nb[2] + bx;
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              if (!dz && !dy && !dx) continue;
              const int dd[3] = {dz, dy, dx};
              Sub s;
              s.rows.nd = 4;
              s.rows.lo[0] = b;
              s.rows.hi[0] = b + 1;
              bool inside = true;
              int nbc[3];
              for (int d = 0; d < 3; ++d) {
                s.rows.lo[d + 1] = dd[d] < 0 ? -h : dd[d] == 0 ? 0 : n[d];
                s.rows.hi[d + 1] = dd[d] < 0 ? 0 : dd[d] == 0 ? n[d] : n[d] + h;
                nbc[d] = bc[d] + dd[d];
                if (nbc[d] < 0 || nbc[d] >= nb[d]) {
                  if (periodic >> d & 1)
                    nbc[d] = (nbc[d] + nb[d]) % nb[d];
                  else
                    inside = false;
                }
              }
              if (!inside) {
                s.kind = SUB_ZERO;
              } else {
                s.kind = SUB_MAP;
                s.w = 1.0;
                std::memset(s.M, 0, sizeof(s.M));
                s.off[0] = ((int64_t)nbc[0] * nb[1] + nbc[1]) * nb[2] + nbc[2];
                for (int d = 0; d < 3; ++d) {
                  s.M[(d + 1) * 4 + (d + 1)] = 1;
                  s.off[d + 1] = -dd[d] * n[d];
                }
              }
              p.subs.push_back(std::move(s));
            }
      }
}

// Block-edge averaging on a vertex-centred cubed sphere (Np points per face
// side).  The boundary point at tangential index t of side `side` of face f
// coincides with the point at t (or Np-1-t when the tangential index runs
// backwards) of the facing side of the neighbour: the same integer links as
// the ghost programs.  Co-located points are merged by union-find; every
// member of a set of k points gets a row with the k members, weight 1/k.
void cs_add_edge_average(Program& p, int64_t Np) {
  const Grid& g = p.grid;
  if (Np < 3) fail(HBC_EINVAL, "edge averaging needs at least 3 points per face side");
  if (g.nd != 3 || g.blocks.size() != 6 || g.blocks[0].data.extent(1) != Np || g.blocks[0].data.extent(2) != Np)
    fail(HBC_EINVAL, "program grid is not the cubed-sphere grid of this Np");
  const int64_t h = -g.blocks[0].full.lo[1];
  const int64_t W = Np + 2 * h;
  const int64_t n = 6 * Np * Np;
  std::vector<int64_t> parent(n);
  std::iota(parent.begin(), parent.end(), 0);
  auto find = [&](int64_t a) {
    while (parent[a] != a) a = parent[a] = parent[parent[a]];
    return a;
  };
  auto point = [&](int f, int side, int64_t t) {
    int64_t j = 0, i = 0;
    if (side == LEFT) { j = t; i = 0; }
    if (side == RIGHT) { j = t; i = Np - 1; }
    if (side == BOTTOM) { j = 0; i = t; }
    if (side == TOP) { j = Np - 1; i = t; }
    return (f * Np + j) * Np + i;
  };
  for (int f = 0; f < 6; ++f)
    for (int side = 0; side < 4; ++side) {
      SideLink L = link(f, side);
      for (int64_t t = 0; t < Np; ++t) {
        const int64_t a = find(point(f, side, t)), b = find(point(L.g, L.gside, L.rev ? Np - 1 - t : t));
        if (a != b) parent[std::max(a, b)] = std::min(a, b);
      }
    }
  std::vector<std::vector<int64_t>> members(n);
  for (int64_t q = 0; q < n; ++q) {
    const int64_t f = q / (Np * Np), j = (q / Np) % Np, i = q % Np;
    if (i != 0 && i != Np - 1 && j != 0 && j != Np - 1) continue;
    members[find(q)].push_back(q);
  }
  // global linear data index of point q over the box [0,6) x [-h, Np+h)^2
  auto lin = [&](int64_t q) {
    const int64_t f = q / (Np * Np), j = (q / Np) % Np, i = q % Np;
    return (f * W + (j + h)) * W + (i + h);
  };
  for (int f = 0; f < 6; ++f) {
    // the face boundary as 4 disjoint boxes: bottom and top rows, then the
    // left and right columns without their ends
    const int64_t boxes[4][4] = {{0, 1, 0, Np}, {Np - 1, Np, 0, Np}, {1, Np - 1, 0, 1}, {1, Np - 1, Np - 1, Np}};
    for (const auto& bx : boxes) {
      DataSub ds;
      ds.rows.nd = 3;
      ds.rows.lo[0] = f;
      ds.rows.hi[0] = f + 1;
      ds.rows.lo[1] = bx[0];
      ds.rows.hi[1] = bx[1];
      ds.rows.lo[2] = bx[2];
      ds.rows.hi[2] = bx[3];
      ds.ptr.push_back(0);
      for (int64_t j = bx[0]; j < bx[1]; ++j)
        for (int64_t i = bx[2]; i < bx[3]; ++i) {
          const int64_t q = (f * Np + j) * Np + i;
          const std::vector<int64_t>& m = members[find(q)];
          if (m.size() < 2) fail(HBC_EINVAL, "internal: a face-boundary point has no co-located copy");
          for (int64_t c : m) {  // members are in ascending point (= cell) order
            ds.cols.push_back(lin(c));
            ds.vals.push_back(1.0 / (double)m.size());
          }
          ds.ptr.push_back((int64_t)ds.cols.size());
        }
      p.dsubs.push_back(std::move(ds));
    }
  }
}

// Wide interpolation rows (Sec. III-B, HOPE's Itp = Agg . Recons): the value
// of edge ghost cell (f, j, i) is a q x q Gauss-Legendre average over the
// cell's square in f's angles of cubic tensor-product Lagrange
// reconstructions on the neighbour face g (4 x 4 nodes per point in g's index
// space, base clamp(floor(s) - 1, 0, N - 4) per direction).  The row is the
// union of the stencils, weights summed, in ascending cell order.  Corner
// ghosts are zero rows.  FP64 geometry on the host, from the integer frames.
void cs_add_quadrature(Program& p, int64_t N, int64_t h, int q, int vector) {
  const Grid& g = p.grid;
  if (N < 4 || h < 1 || 2 * h > N)
    fail(HBC_EINVAL, "cubed sphere needs N >= 4 and 1 <= h <= N/2 (deeper ghost layers leave the face's gnomonic chart)");
  if (g.nd != 3 || g.blocks.size() != 6 || g.blocks[0].data.extent(1) != N ||
      g.blocks[0].full.lo[1] != -h || g.blocks[0].full.hi[1] != N + h)
    fail(HBC_EINVAL, "program grid is not the cubed-sphere grid of this N and h");
  // Gauss-Legendre nodes (in cell widths, on [-1/2, 1/2]) and weights (sum 1)
  std::vector<double> xn, wn;
  if (q == 1) {
    xn = {0.0};
    wn = {1.0};
  } else if (q == 2) {
    const double a = 0.5 / std::sqrt(3.0);
    xn = {-a, a};
    wn = {0.5, 0.5};
  } else if (q == 3) {
    const double a = 0.5 * std::sqrt(0.6);
    xn = {-a, 0.0, a};
    wn = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
  } else {
    fail(HBC_EINVAL, "quadrature order must be 1, 2 or 3");
  }
  const double D = M_PI / (2.0 * (double)N);
  const double Q = M_PI / 4.0;
  const int64_t W = N + 2 * h;
  auto lin = [&](int64_t f, int64_t j, int64_t i) { return (f * W + (j + h)) * W + (i + h); };
  auto lag4 = [&](double s, int64_t& base, double* w) {
    base = (int64_t)std::floor(s) - 1;
    base = base < 0 ? 0 : (base > N - 4 ? N - 4 : base);
    const double d0 = s - base, d1 = s - (base + 1), d2 = s - (base + 2), d3 = s - (base + 3);
    w[0] = -d1 * d2 * d3 / 6.0;
    w[1] = d0 * d2 * d3 / 2.0;
    w[2] = -d0 * d1 * d3 / 2.0;
    w[3] = d0 * d1 * d2 / 6.0;
  };
  for (int f = 0; f < 6; ++f) {
    for (int side = 0; side < 4; ++side) {
      SideLink L = link(f, side);
      Sub s;
      s.kind = SUB_CSR;
      s.rows.nd = 3;
      s.rows.lo[0] = f;
      s.rows.hi[0] = f + 1;
      if (side == LEFT) { s.rows.lo[1] = 0; s.rows.hi[1] = N; s.rows.lo[2] = -h; s.rows.hi[2] = 0; }
      if (side == RIGHT) { s.rows.lo[1] = 0; s.rows.hi[1] = N; s.rows.lo[2] = N; s.rows.hi[2] = N + h; }
      if (side == BOTTOM) { s.rows.lo[1] = -h; s.rows.hi[1] = 0; s.rows.lo[2] = 0; s.rows.hi[2] = N; }
      if (side == TOP) { s.rows.lo[1] = N; s.rows.hi[1] = N + h; s.rows.lo[2] = 0; s.rows.hi[2] = N; }
      s.rot = vector ? rot_code(L.rot) : 0;
      if (s.rot < 0) fail(HBC_EINVAL, "internal: face rotation is not a signed permutation");
      const V3 cf = FR[f][0], e1f = FR[f][1], e2f = FR[f][2];
      const V3 cg = FR[L.g][0], e1g = FR[L.g][1], e2g = FR[L.g][2];
      s.ptr.push_back(0);
      for (int64_t j = s.rows.lo[1]; j < s.rows.hi[1]; ++j)
        for (int64_t i = s.rows.lo[2]; i < s.rows.hi[2]; ++i) {
          std::map<int64_t, double> acc;
          for (size_t b = 0; b < xn.size(); ++b)
            for (size_t a = 0; a < xn.size(); ++a) {
              const double ta = std::tan(-Q + ((double)i + 0.5 + xn[a]) * D);
              const double tb = std::tan(-Q + ((double)j + 0.5 + xn[b]) * D);
              // P = c_f + ta e1_f + tb e2_f, seen from g
              const double Px = cf.x + ta * e1f.x + tb * e2f.x, Py = cf.y + ta * e1f.y + tb * e2f.y,
                           Pz = cf.z + ta * e1f.z + tb * e2f.z;
              const double pc = Px * cg.x + Py * cg.y + Pz * cg.z;
              const double ag = std::atan((Px * e1g.x + Py * e1g.y + Pz * e1g.z) / pc);
              const double bg = std::atan((Px * e2g.x + Py * e2g.y + Pz * e2g.z) / pc);
              const double si = (ag + Q) / D - 0.5, sj = (bg + Q) / D - 0.5;
              int64_t bj, bi;
              double wj[4], wi[4];
              lag4(sj, bj, wj);
              lag4(si, bi, wi);
              const double wq = wn[a] * wn[b];
              for (int u = 0; u < 4; ++u)
                for (int v = 0; v < 4; ++v) acc[lin(L.g, bj + u, bi + v)] += wq * wj[u] * wi[v];
            }
          for (const auto& kv : acc) {
            s.cols.push_back(kv.first);
            s.vals.push_back(kv.second);
          }
          s.ptr.push_back((int64_t)s.cols.size());
        }
      p.subs.push_back(std::move(s));
    }
    const int64_t lo[2] = {-h, N}, hi[2] = {0, N + h};
    for (int a = 0; a < 2; ++a)
      for (int c = 0; c < 2; ++c) {
        Sub z;
        z.kind = SUB_ZERO;
        z.rows.nd = 3;
        z.rows.lo[0] = f;
        z.rows.hi[0] = f + 1;
        z.rows.lo[1] = lo[a];
        z.rows.hi[1] = hi[a];
        z.rows.lo[2] = lo[c];
        z.rows.hi[2] = hi[c];
        p.subs.push_back(z);
      }
  }
}

}  // namespace hbc
