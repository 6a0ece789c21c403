// Host-side exercise of the C ABI for the sanitizer test (built with
// AddressSanitizer and UndefinedBehaviorSanitizer, no device code): every
// program builder, host-only plan compiles, row queries, new sub-vector
// values, tuning and error paths; then the same scenario with the k-th host
// allocation made to fail (operator new throws), for a sweep of k: every call
// must return HBC_OK or HBC_ENOMEM, and nothing may leak (the leak checker
// runs at exit).  Exit status 0 when every check holds.
#include <cstdio>
#include <cstdlib>
#include <new>
#include <vector>

#include "hbc.h"

static long g_fail_at = -1;  // allocation number that throws, or -1
static long g_count = 0;     // allocations since the counter was armed
static bool g_failed = false;

void* operator new(std::size_t n) {
  if (g_fail_at >= 0 && ++g_count == g_fail_at) {
    g_failed = true;
    throw std::bad_alloc();
  }
  void* p = std::malloc(n ? n : 1);
  if (!p) throw std::bad_alloc();
  return p;
}
void* operator new[](std::size_t n) { return operator new(n); }
// the nothrow forms (std::stable_sort's temporary buffer) pair with the same delete
void* operator new(std::size_t n, const std::nothrow_t&) noexcept {
  try {
    return operator new(n);
  } catch (...) {
    return nullptr;
  }
}
void* operator new[](std::size_t n, const std::nothrow_t& t) noexcept { return operator new(n, t); }
void operator delete(void* p) noexcept { std::free(p); }
void operator delete[](void* p) noexcept { std::free(p); }
void operator delete(void* p, std::size_t) noexcept { std::free(p); }
void operator delete[](void* p, std::size_t) noexcept { std::free(p); }

static int g_errors = 0;

// OK, or ENOMEM while an allocation failure is armed; anything else is an error
#define CALL(x)                                                                                     \
  do {                                                                                              \
    const int rc_ = (x);                                                                            \
    if (rc_ == HBC_ENOMEM && g_fail_at >= 0) goto done;                                             \
    if (rc_ != HBC_OK) {                                                                            \
      std::fprintf(stderr, "%s:%d %s -> %d (%s)\n", __FILE__, __LINE__, #x, rc_, hbc_last_error()); \
      ++g_errors;                                                                                   \
      goto done;                                                                                    \
    }                                                                                               \
  } while (0)

#define EXPECT(x, code)                                                                             \
  do {                                                                                              \
    const int rc_ = (x);                                                                            \
    if (rc_ == HBC_ENOMEM && g_fail_at >= 0) goto done;                                             \
    if (rc_ != (code)) {                                                                            \
      std::fprintf(stderr, "%s:%d %s -> %d, wanted %d\n", __FILE__, __LINE__, #x, rc_, (code));    \
      ++g_errors;                                                                                   \
      goto done;                                                                                    \
    }                                                                                               \
  } while (0)

// the driver's own buffers, allocated before any failure is armed
struct Buffers {
  static constexpr int64_t N = 12, h = 3, I = 8;
  std::vector<int32_t> base;
  std::vector<double> w, b, b2, vals;
  std::vector<int64_t> cols;
  Buffers() : base(h * N), w(4 * h * N), b(N * h * I, 0.5), b2(N * h * I, -1.5), vals(64), cols(64) {
    const double ws[4] = {-0.0625, 0.5625, 0.5625, -0.0625};
    for (int64_t k = 0; k < h; ++k)
      for (int64_t t = 0; t < N; ++t) {
        base[k * N + t] = (int32_t)(t < 1 ? 0 : (t - 1 > N - 4 ? N - 4 : t - 1));
        for (int m = 0; m < 4; ++m) w[(k * N + t) * 4 + m] = ws[m];
      }
  }
};

static void scenario(Buffers& B) {
  const int64_t N = Buffers::N, h = Buffers::h, I = Buffers::I;
  hbc_grid *g = nullptr, *gc = nullptr, *gq = nullptr, *ge = nullptr, *gs = nullptr;
  hbc_program *p = nullptr, *pc = nullptr, *pq = nullptr, *pe = nullptr, *ps = nullptr, *pf = nullptr;
  hbc_plan *pl = nullptr, *plc = nullptr, *plq = nullptr, *ple = nullptr, *pls = nullptr, *plf = nullptr;
  hbc_stats st;
  hbc_tune tu;
  int32_t sid = -1, nnz = 0, kind = 0, rot = 0, blk = 0;
  double bv = 0;
  {
    // cubed sphere, Lagrange rows with rotation, a sub-vector, host-only plan
    CALL(hbc_cs_grid_create(N, h, &g));
    CALL(hbc_program_create(g, &p));
    CALL(hbc_cs_program_add(p, N, h, HBC_CS_LAGRANGE, 1, B.base.data(), B.w.data()));
    hbc_box box{};
    box.lo[0] = 0, box.lo[1] = 0, box.lo[2] = -h;
    box.hi[0] = 1, box.hi[1] = N, box.hi[2] = 0;
    CALL(hbc_program_add_vector(p, &box, I, B.b.data(), &sid));
    hbc_layout lay{I, HBC_POINT_MAJOR, 2, 4, 2};
    CALL(hbc_plan_create(p, &lay, HBC_F64, HBC_PLAN_HOST_ONLY, &pl));
    CALL(hbc_plan_stats(pl, &st));
    for (int64_t c = 0; c < 6 * (N + 2 * h) * (N + 2 * h); c += 37)
      CALL(hbc_plan_row(pl, c, c % I, 64, B.cols.data(), B.vals.data(), &nnz, &bv, &kind, &rot));
    CALL(hbc_plan_set_vector(pl, sid, B.b2.data(), nullptr));
    CALL(hbc_plan_get_tune(pl, &tu));
    tu.rows_per_tile = 5;
    CALL(hbc_plan_set_tune(pl, &tu));
    // device calls on a host-only plan are refused without touching a device
    double dummy[2];
    EXPECT(hbc_apply(pl, dummy, 2, nullptr), HBC_EINVAL);
    // consumers compiled on the host-only plan: the cross and the 9-point box
    // (the line walk's order), a skewed stencil (the general order); applies
    // refused, an offset reaching past the halo refused
    {
      const int64_t cross[15] = {0, 0, 0, 0, 1, 0, 0, -1, 0, 0, 0, 1, 0, 0, -1};
      const int64_t skew[12] = {0, 2, -1, 0, 0, 0, 0, -1, 2, 0, -3, 3};
      int64_t box9[27];
      double w9[9];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          box9[3 * (3 * a + b)] = 0, box9[3 * (3 * a + b) + 1] = a - 1, box9[3 * (3 * a + b) + 2] = 1 - b;
          w9[3 * a + b] = 0.5 * (a + 1) - b;
        }
      const double wc[5] = {-4, 1, 1, 1, 1}, ws[4] = {0.25, -1.5, 2.0, 0.75};
      const int64_t far[3] = {0, 4, 0};
      int64_t nbr = 0, nbe = 0;
      hbc_consumer* cs = nullptr;
      CALL(hbc_consumer_create(pl, 5, cross, wc, &cs));
      const int st1 = hbc_consumer_stats(cs, &nbr, &nbe);
      const int ap1 = hbc_consumer_apply(cs, dummy, 2, dummy, 2, 1, nullptr);
      hbc_consumer_destroy(cs);
      CALL(st1);
      EXPECT(ap1, HBC_EINVAL);
      CALL(hbc_consumer_create(pl, 9, box9, w9, &cs));
      hbc_consumer_destroy(cs);
      CALL(hbc_consumer_create(pl, 4, skew, ws, &cs));
      hbc_consumer_destroy(cs);
      cs = nullptr;
      EXPECT(hbc_consumer_create(pl, 1, far, wc, &cs), HBC_EINVAL);
    }
    EXPECT(hbc_plan_create(nullptr, &lay, HBC_F64, HBC_PLAN_HOST_ONLY, &plf), HBC_EINVAL);
    hbc_layout bad{0, HBC_POINT_MAJOR, 0, 0, 0};
    EXPECT(hbc_plan_create(p, &bad, HBC_F64, HBC_PLAN_HOST_ONLY, &plf), HBC_EINVAL);
    // the same program with a consumer footprint, FP32, plane-major
    CALL(hbc_program_create(g, &pf));
    CALL(hbc_cs_program_add(pf, N, h, HBC_CS_SYNC, 1, nullptr, nullptr));
    const int64_t cross[15] = {0, 0, 0, 0, 1, 0, 0, -1, 0, 0, 0, 1, 0, 0, -1};
    CALL(hbc_program_set_consumer(pf, 5, cross));
    hbc_layout lay2{I, HBC_PLANE_MAJOR, 2, 4, 2};
    CALL(hbc_plan_create(pf, &lay2, HBC_F32, HBC_PLAN_HOST_ONLY, &plf));
    {
      hbc_consumer* cp = nullptr;
      EXPECT(hbc_consumer_create(plf, 5, cross, nullptr, &cp), HBC_EINVAL);  // no weights
      const double wc[5] = {-4, 1, 1, 1, 1};
      EXPECT(hbc_consumer_create(plf, 5, cross, wc, &cp), HBC_EUNSUPPORTED);  // plane-major
    }
    // Cartesian blocks with a one-cell halo, one periodic direction
    const int32_t nb[3] = {2, 2, 2};
    const int64_t n[3] = {4, 4, 5};
    CALL(hbc_cart_grid_create(nb, n, 1, &gc));
    CALL(hbc_program_create(gc, &pc));
    CALL(hbc_cart_program_add_halo(pc, nb, n, 1, 4));
    hbc_layout lay3{1, HBC_POINT_MAJOR, 0, 0, 0};
    CALL(hbc_plan_create(pc, &lay3, HBC_F64, HBC_PLAN_HOST_ONLY, &plc));
    // wide quadrature rows with rotation
    CALL(hbc_cs_grid_create(8, 2, &gq));
    CALL(hbc_program_create(gq, &pq));
    CALL(hbc_cs_program_add_quadrature(pq, 8, 2, 2, 1));
    hbc_layout lay4{6, HBC_POINT_MAJOR, 2, 2, 2};
    CALL(hbc_plan_create(pq, &lay4, HBC_F64, HBC_PLAN_HOST_ONLY, &plq));
    // block-edge averaging on a vertex-centred cube (data rows)
    CALL(hbc_cs_grid_create(9, 1, &ge));
    CALL(hbc_program_create(ge, &pe));
    CALL(hbc_cs_program_add(pe, 9, 1, HBC_CS_SYNC, 0, nullptr, nullptr));
    CALL(hbc_cs_program_add_edge_average(pe, 9));
    hbc_layout lay5{4, HBC_POINT_MAJOR, 0, 0, 0};
    CALL(hbc_plan_create(pe, &lay5, HBC_F64, HBC_PLAN_HOST_ONLY, &ple));
    // stepped slices: a staggered line, mirror map on the left, zeros elsewhere
    const int64_t lo[2] = {0, 0}, hi[2] = {1, 41};
    CALL(hbc_grid_create(2, lo, hi, &gs));
    const hbc_slice full[2] = {{0, 1, 1}, {1, 41, 2}}, data[2] = {{0, 1, 1}, {5, 37, 2}};
    CALL(hbc_grid_add_block(gs, full, data, &blk));
    CALL(hbc_program_create(gs, &ps));
    hbc_box lb{};
    lb.lo[0] = 0, lb.lo[1] = 1, lb.hi[0] = 1, lb.hi[1] = 5;
    const int64_t M[4] = {1, 0, 0, -1}, off[2] = {0, 10};
    CALL(hbc_program_add_map(ps, &lb, M, off, 1.0, nullptr, &sid));
    CALL(hbc_program_add_zero_rest(ps, 0, &sid));
    hbc_layout lay6{3, HBC_POINT_MAJOR, 0, 0, 0};
    CALL(hbc_plan_create(ps, &lay6, HBC_F64, HBC_PLAN_HOST_ONLY, &pls));
    CALL(hbc_plan_stats(pls, &st));
  }
done:
  hbc_plan_destroy(pl);
  hbc_plan_destroy(plf);
  hbc_plan_destroy(plc);
  hbc_plan_destroy(plq);
  hbc_plan_destroy(ple);
  hbc_plan_destroy(pls);
  hbc_program_destroy(p);
  hbc_program_destroy(pf);
  hbc_program_destroy(pc);
  hbc_program_destroy(pq);
  hbc_program_destroy(pe);
  hbc_program_destroy(ps);
  hbc_grid_destroy(g);
  hbc_grid_destroy(gc);
  hbc_grid_destroy(gq);
  hbc_grid_destroy(ge);
  hbc_grid_destroy(gs);
}

int main() {
  Buffers B;
  scenario(B);  // the plain run: every call succeeds
  if (g_errors) return 1;
  // count the scenario's allocations, then fail each of a sweep of them
  g_fail_at = 0x7fffffffffffffffL;
  g_count = 0;
  scenario(B);
  const long total = g_count;
  long runs = 0, hit = 0;
  for (long k = 1; k <= total; k += (k < 3000 ? 1 : 11)) {
    g_fail_at = k;
    g_count = 0;
    g_failed = false;
    scenario(B);
    ++runs;
    hit += g_failed ? 1 : 0;
    if (g_errors) {
      std::fprintf(stderr, "allocation %ld of %ld failing gave an error other than HBC_ENOMEM\n", k, total);
      return 1;
    }
  }
  g_fail_at = -1;
  std::printf("allocations %ld, failure runs %ld, failures injected %ld\n", total, runs, hit);
  return hit > 0 ? 0 : 1;
}
