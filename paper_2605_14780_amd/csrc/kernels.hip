// HIP kernels for gfx950 (CDNA4, wave64) and their launchers.
//
// The apply is a bandwidth-bound sparse gather/scatter (Sec. III-B: every BC
// kind is a row of y = A x + b), so there is no MFMA here: the work is laid
// out so that every wavefront reads and writes contiguous runs of the field.
//   point-major fields (value (cell, l) at cell*inner + l): the lanes of a
//     row walk its inner values with 16-byte accesses, so a ghost row is one
//     contiguous write and each source cell one contiguous read;
//   plane-major fields (l*ncells + cell): lanes walk consecutive rows of a
//     segment box, which are consecutive cells along the box's last dimension.
// Each workgroup takes tiles of one segment (a disjoint box of rows of one
// kind, Sec. IV-C), so the kind switch is uniform per workgroup.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <cxxabi.h>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <type_traits>
#include <vector>

#include "device.hpp"

namespace hbc {

#define HIP_CHECK(x)                                                                           \
  do {                                                                                         \
    hipError_t e_ = (x);                                                                       \
    if (e_ != hipSuccess) fail(HBC_EHIP, std::string(#x) + ": " + hipGetErrorString(e_));      \
  } while (0)

// ---- per-launch descriptor of one plan applied to one field ---------------------------
struct PlanDesc {
  void* field;
  const DevSeg* segs;
  const int32_t* ell_col;
  const void* ell_val;
  const int64_t* csr_ptr;
  const int32_t* csr_col;
  const void* csr_val;
  const void* bval;
  int64_t cs, ls;  // element offset of (cell, l) = cell*cs + l*ls
  int64_t inner;
  int64_t vec_lo, vec_stride, vec_len;
  int32_t lpr_shift;  // log2 lanes per row
  int32_t vec;        // elements per lane access
  int32_t chunked;    // point-major: each row group walks a contiguous run of rows
  int32_t nt;         // results go out with non-temporal stores (rows of >= 128 bytes)
  int32_t unroll;     // accesses of vec elements per lane and row (point-major)
  int32_t general;    // the row tiles hold general ELL/CSR rows
  int32_t ua;         // point-major rows as 16-byte vectors on 4-byte (FP32) or 8-byte (FP64)
                      // boundaries, the last one ending at the row's end (see rt_tile)
  const int32_t* row_dst;  // point-major row tables
  const int32_t* row_src;
};

struct AdjDesc {
  const int64_t* src;
  const int64_t* ptr;
  const int64_t* ghost;
  const void* w;
  const int32_t* rot;
  const int32_t* cnt;  // entries per source
  const int32_t* fg;   // fixed-width entries: ghost cell, weight, rotation at k*aw + m
  const void* fw;
  const int8_t* frot;
  int32_t aw;
};

template <typename T, int V>
struct Pack {
  T v[V];
};

// UA: p is aligned only to the element size (vector accesses on element
// boundaries are legal for global memory on gfx9 and later).
template <typename T, int V, bool UA = false>
__device__ __forceinline__ Pack<T, V> ldv(const T* p) {
  Pack<T, V> r;
  if constexpr (V == 1) {
    r.v[0] = *p;
  } else {
    typedef T vt __attribute__((ext_vector_type(V), aligned(UA ? sizeof(T) : V * sizeof(T))));
    vt x = *reinterpret_cast<const vt*>(p);
#pragma unroll
    for (int i = 0; i < V; ++i) r.v[i] = x[i];
  }
  return r;
}

// Results that no later access in the same kernel reads may go out as
// non-temporal stores (streamed past the caches rather than allocated in
// them).  That pays for whole rows of 128 bytes or more; for short scattered
// rows the caches merge partial lines and plain stores are faster.
template <typename T, int V, bool NT, bool UA = false>
__device__ __forceinline__ void stv(T* p, const Pack<T, V>& r) {
  if constexpr (V == 1) {
    if (NT)
      __builtin_nontemporal_store(r.v[0], p);
    else
      *p = r.v[0];
  } else {
    typedef T vt __attribute__((ext_vector_type(V), aligned(UA ? sizeof(T) : V * sizeof(T))));
    vt x;
#pragma unroll
    for (int i = 0; i < V; ++i) x[i] = r.v[i];
    if (NT)
      __builtin_nontemporal_store(x, reinterpret_cast<vt*>(p));
    else
      *reinterpret_cast<vt*>(p) = x;
  }
}

// Raw buffer accesses: a store at an offset past the resource's range is
// dropped by the hardware, so a lane that stores nothing can still issue the
// instruction (ranges stay below 2 GiB, so BUF_OOB is past every one).
constexpr uint32_t BUF_OOB = 0x80000000u;
constexpr int32_t BUF_RSRC_WORD3 = 0x00020000;  // raw buffer, 32-bit data format

// Store of one pack through a buffer resource (dropped where off is out of range).
template <typename T, int V, bool NT>
__device__ __forceinline__ void stv_buf(const Pack<T, V>& p, __amdgpu_buffer_rsrc_t r, uint32_t off) {
  constexpr int AUX = NT ? 2 : 0;  // non-temporal
  constexpr int BYTES = (int)sizeof(T) * V;
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  if constexpr (BYTES == 16) {
    typedef T tv __attribute__((ext_vector_type(V)));
    tv v;
#pragma unroll
    for (int i = 0; i < V; ++i) v[i] = p.v[i];
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, off, 0, AUX);
  } else if constexpr (BYTES == 8 && V == 1) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, p.v[0]), r, off, 0, AUX);
  } else if constexpr (BYTES == 8) {
    typedef T tv __attribute__((ext_vector_type(V)));
    tv v;
#pragma unroll
    for (int i = 0; i < V; ++i) v[i] = p.v[i];
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, AUX);
  } else {
    static_assert(BYTES == 4, "pack of 4, 8 or 16 bytes");
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, p.v[0]), r, off, 0, AUX);
  }
}

// Source inner slot of output slot l under rotation code `rot` (see rot_code):
// component a of the vector takes sign_a * component p(a) of the source.
template <typename T>
__device__ __forceinline__ int64_t rot_slot(const PlanDesc& d, int rot, int64_t l, T& sign) {
  sign = T(1);
  if (rot == 0 || d.vec_len == 0) return l;
  int64_t off = l - d.vec_lo;
  int a;
  if (off >= 0 && off < d.vec_len) {
    a = 0;
  } else if (off >= d.vec_stride && off < d.vec_stride + d.vec_len) {
    a = 1;
    off -= d.vec_stride;
  } else {
    return l;
  }
  const int p = (rot & 1) ? 1 - a : a;
  if (rot & (2 << a)) sign = T(-1);
  return d.vec_lo + p * d.vec_stride + off;
}

// Plane-major tile: rows [row0, row0 + nrows) of segment s, all inner values.
// Consecutive threads take consecutive rows (neighbouring ghost cells are
// neighbours in every plane), the lpr thread sets of a workgroup take planes
// l = lane, lane + lpr, ...; a thread reads its row's columns and weights
// once and then works through its planes PB at a time, all loads of the PB
// planes issued before any arithmetic or store.
constexpr int PB = 8;

template <typename T>
__device__ __forceinline__ void run_tile_pm(const PlanDesc& d, const DevSeg& s, int64_t row0, int nrows,
                                            bool zero_only, int tid, int nthr) {
  const int lpr = 1 << d.lpr_shift;
  const int rp = nthr >> d.lpr_shift;  // rows per pass
  const int rsub = tid % rp, lane = tid / rp;
  const int64_t nvec = d.inner;
  T* __restrict__ f = static_cast<T*>(d.field);
  const int kind = zero_only ? (int)SEG_ZERO : s.kind;
  const bool add_b = !zero_only && s.has_b;
  const bool narrow = kind == SEG_ELL && s.width <= 4;
  for (int r = rsub; r < nrows; r += rp) {
    const int64_t row = row0 + r;
    uint32_t q = (uint32_t)row;
    int64_t dst = s.dst_base, src = s.src_base;
    // every SEG_MAXD dimension (unused ones have extent 1 and stride 0), so
    // that the segment's arrays are read at constant indices, from registers
#pragma unroll
    for (int k = SEG_MAXD - 1; k >= 0; --k) {
      const uint32_t e = (uint32_t)s.ext[k];
      const uint32_t c = q % e;
      q /= e;
      dst += (int64_t)c * s.dst_stride[k];
      src += (int64_t)c * s.src_stride[k];
    }
    const T* bp = nullptr;
    if (add_b) bp = static_cast<const T*>(d.bval) + s.brow + row * s.b_inner;
    int32_t col[4] = {-1, -1, -1, -1};
    T wt[4] = {T(0), T(0), T(0), T(0)};
    if (narrow) {
      const int64_t e0 = s.tab + row * s.width;
#pragma unroll
      for (int m = 0; m < 4; ++m)
        if (m < s.width) {
          col[m] = d.ell_col[e0 + m];
          wt[m] = static_cast<const T*>(d.ell_val)[e0 + m];
        }
    }
    for (int64_t v0 = lane; v0 < nvec; v0 += (int64_t)lpr * PB) {
      int64_t l[PB], sl[PB];
      T sign[PB];
      bool ok[PB];
#pragma unroll
      for (int u = 0; u < PB; ++u) {
        const int64_t v = v0 + (int64_t)u * lpr;
        ok[u] = v < nvec;
        l[u] = ok[u] ? v : v0;
        sign[u] = T(1);
        sl[u] = (kind == SEG_MAP || kind == SEG_ELL || kind == SEG_CSR) ? rot_slot<T>(d, s.rot, l[u], sign[u]) : l[u];
      }
      T y[PB];
      if (kind == SEG_MAP) {
        T x[PB];
#pragma unroll
        for (int u = 0; u < PB; ++u) x[u] = f[src * d.cs + sl[u] * d.ls];
#pragma unroll
        for (int u = 0; u < PB; ++u) y[u] = (T(s.w) * sign[u]) * x[u];
      } else if (narrow) {
        T x[PB][4];
#pragma unroll
        for (int u = 0; u < PB; ++u)
#pragma unroll
          for (int m = 0; m < 4; ++m) x[u][m] = col[m] >= 0 ? f[(int64_t)col[m] * d.cs + sl[u] * d.ls] : T(0);
#pragma unroll
        for (int u = 0; u < PB; ++u) {
          T acc = T(0);
          bool first = true;
#pragma unroll
          for (int m = 0; m < 4; ++m)
            if (col[m] >= 0) {
              acc = first ? wt[m] * x[u][m] : fma(wt[m], x[u][m], acc);
              first = false;
            }
          y[u] = sign[u] * acc;
        }
      } else if (kind == SEG_ELL || kind == SEG_CSR) {
        int64_t e0, e1;
        const int32_t* cols;
        const T* vals;
        if (kind == SEG_ELL) {
          e0 = s.tab + row * s.width;
          e1 = e0 + s.width;
          cols = d.ell_col;
          vals = static_cast<const T*>(d.ell_val);
        } else {
          e0 = d.csr_ptr[s.tab + row];
          e1 = d.csr_ptr[s.tab + row + 1];
          cols = d.csr_col;
          vals = static_cast<const T*>(d.csr_val);
        }
        T acc[PB];
#pragma unroll
        for (int u = 0; u < PB; ++u) acc[u] = T(0);
        bool first = true;
        for (int64_t e = e0; e < e1; ++e) {
          const int32_t c = cols[e];
          if (c < 0) continue;
          const T w = vals[e];
          T x[PB];
#pragma unroll
          for (int u = 0; u < PB; ++u) x[u] = f[(int64_t)c * d.cs + sl[u] * d.ls];
#pragma unroll
          for (int u = 0; u < PB; ++u) acc[u] = first ? w * x[u] : fma(w, x[u], acc[u]);
          first = false;
        }
#pragma unroll
        for (int u = 0; u < PB; ++u) y[u] = sign[u] * acc[u];
      } else {  // zero rows, or b-only rows
#pragma unroll
        for (int u = 0; u < PB; ++u) y[u] = T(0);
      }
      if (add_b) {
#pragma unroll
        for (int u = 0; u < PB; ++u) {
          const T bb = s.b_inner == 1 ? bp[0] : bp[l[u]];
          y[u] = (kind == SEG_VEC) ? bb : y[u] + bb;
        }
      }
#pragma unroll
      for (int u = 0; u < PB; ++u)
        if (ok[u]) f[dst * d.cs + l[u] * d.ls] = y[u];
    }
  }
}

// Point-major tile over the per-row tables: the lanes of a row group cover
// the inner values of one row with 16-byte accesses.  A row group works
// through its rows in batches of RB: destination cells, columns and weights
// of the batch are read first, then every source load of the batch is issued
// before any arithmetic or store, so a lane keeps up to 4*RB independent
// loads in flight; repeated sources of neighbouring rows hit in L1/L2.  With
// groups of >= CHUNK_LPR lanes a row group takes a contiguous run of rows,
// otherwise rows are dealt round-robin so that neighbouring lanes write
// neighbouring cells.
// RB (rows per batch of a row group) is rows_per_batch(lanes per row): 2 for
// rows of >= 128 lanes (>= 2 KiB: the batch is already many loads, and short
// tiles keep more workgroups in flight), else 4.

// U > 1: a lane carries U accesses of V elements per row, lpr apart (rows
// whose length is not a multiple of a 16-byte vector still keep 16 bytes of
// loads per lane and source in flight, and every access stays coalesced).
// KM: the row kinds the tile list may hold besides copies, zero and b rows:
// bit 0 the 4-wide Lagrange rows, bit 1 general ELL/CSR rows.  Paths of
// absent kinds are compiled out (their registers would lower the occupancy of
// every other kind).
// KM_SEQFB: Lagrange row batches whose windows do not slide go row by row
// (see the ELL path).
constexpr int KM_ELL4 = 1, KM_GENERAL = 2, KM_UNAL = 4, KM_SEQFB = 8;
template <typename T, int V, int U, bool NT, int RB, int KM>
__device__ __forceinline__ void rt_tile(const PlanDesc& d, const RowTile& tl, bool zero_only) {
  const int lpr = 1 << d.lpr_shift;
  const int ngroups = (int)blockDim.x >> d.lpr_shift;
  const int grp = (int)threadIdx.x >> d.lpr_shift;
  const int lane = (int)threadIdx.x & (lpr - 1);
  // KM_UNAL: rows whose length is not a multiple of V go as ceil(inner / V)
  // vectors on element boundaries, the last one moved back to end at the
  // row's end.  The slots it shares with the vector before it get the same
  // value twice (every slot's arithmetic is independent of the vector it
  // sits in), and stores reach only ghost rows, which no load reads.
  constexpr bool UA = (KM & KM_UNAL) != 0;
  const int64_t nvec = UA ? (d.inner + V - 1) / V : d.inner / V;
  T* __restrict__ f = static_cast<T*>(d.field);
  const int kind = zero_only ? (int)SEG_ZERO : tl.kind;
  const bool with_b = !zero_only && tl.has_b;
  const int nrows = tl.nrows;
  int rb, re, rs;
  if (d.chunked) {
    const int ch = (nrows + ngroups - 1) / ngroups;
    rb = grp * ch;
    re = min(nrows, rb + ch);
    rs = 1;
  } else {
    rb = grp;
    re = nrows;
    rs = ngroups;
  }
  if (rb >= re) return;
  const int last = rb + ((re - 1 - rb) / rs) * rs;
  const int32_t* __restrict__ rdst = d.row_dst + tl.row_begin;
  const int32_t* __restrict__ rsrc = d.row_src + tl.row_begin;
  const bool ell4 = (KM & KM_ELL4) && kind == SEG_ELL && tl.width == 4 && !(tl.flags & SEGF_ELL_PADDED);
  const T* __restrict__ bt = static_cast<const T*>(d.bval) + tl.brow;
  const bool rotates = kind == SEG_MAP || kind == SEG_ELL || kind == SEG_CSR;
  for (int64_t v0 = lane; v0 < nvec; v0 += (int64_t)lpr * U) {
    int64_t l[U], sl[U];
    T sign[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t v = v0 + (int64_t)u * lpr;
      ok[u] = v < nvec;
      l[u] = (ok[u] ? v : v0) * V;  // a spare access repeats a valid one and is not stored
      if (UA) l[u] = min(l[u], d.inner - V);
      sign[u] = T(1);
      sl[u] = rotates ? rot_slot<T>(d, tl.rot, l[u], sign[u]) : l[u];
    }
    for (int r = rb; r < re; r += RB * rs) {
      int rr[RB];
      int64_t dst[RB];
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        rr[q] = min(r + q * rs, last);
        dst[q] = rdst[rr[q]];
      }
      Pack<T, V> y[RB][U];
      if (kind == SEG_MAP) {
        Pack<T, V> x[RB][U];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
          const T* src = f + (int64_t)rsrc[rr[q]] * d.cs;
#pragma unroll
          for (int u = 0; u < U; ++u) x[q][u] = ldv<T, V, UA>(src + sl[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const T wt = T(tl.w) * sign[u];
#pragma unroll
          for (int q = 0; q < RB; ++q)
#pragma unroll
            for (int i = 0; i < V; ++i) y[q][u].v[i] = wt * x[q][u].v[i];
        }
      } else if (ell4) {
        const int32_t* __restrict__ cb = d.ell_col + tl.tab;
        const T* __restrict__ vb = static_cast<const T*>(d.ell_val) + tl.tab;
        int32_t c[RB][4];
        T wt[RB][4];
#pragma unroll
        for (int q = 0; q < RB; ++q)
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            c[q][m] = cb[rr[q] * 4 + m];
            wt[q][m] = vb[rr[q] * 4 + m];
          }
        // Consecutive rows along a face-edge strip usually read a window
        // that slides by one cell of the neighbour's grid line:
        // c[q][m] = c[0][0] + (q + m) * dl.  Then the batch needs RB + 3
        // distinct sources instead of 4 * RB.
        const int32_t c00 = c[0][0];
        const int32_t dl = c[0][1] - c[0][0];
        bool slide = dl != 0;
#pragma unroll
        for (int q = 0; q < RB; ++q)
#pragma unroll
          for (int m = 0; m < 4; ++m) slide = slide && (c[q][m] == c00 + (q + m) * dl);
        if (slide) {
          Pack<T, V> w[RB + 3][U];
#pragma unroll
          for (int j = 0; j < RB + 3; ++j) {
            const T* src = f + (int64_t)(c00 + j * dl) * d.cs;
#pragma unroll
            for (int u = 0; u < U; ++u) w[j][u] = ldv<T, V, UA>(src + sl[u]);
          }
#pragma unroll
          for (int q = 0; q < RB; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
              for (int i = 0; i < V; ++i) {
                T a = wt[q][0] * w[q][u].v[i];
                a = fma(wt[q][1], w[q + 1][u].v[i], a);
                a = fma(wt[q][2], w[q + 2][u].v[i], a);
                a = fma(wt[q][3], w[q + 3][u].v[i], a);
                y[q][u].v[i] = sign[u] * a;
              }
        } else if constexpr ((KM & KM_SEQFB) != 0) {
          // the windows do not slide (a run restarts inside the batch, or the
          // group's rows end before the batch does): row by row, so that this
          // path holds one row's sources rather than the batch's, and the
          // kernel (whose registers are those of its largest path) keeps more
          // waves resident
#pragma unroll
          for (int q = 0; q < RB; ++q) {
            if (q > 0 && rr[q] == rr[q - 1]) {
              // past the group's last row (clamped to it): its value, no loads
#pragma unroll
              for (int u = 0; u < U; ++u) y[q][u] = y[q - 1][u];
            } else {
              Pack<T, V> x[4][U];
#pragma unroll
              for (int m = 0; m < 4; ++m) {
                const T* src = f + (int64_t)c[q][m] * d.cs;
#pragma unroll
                for (int u = 0; u < U; ++u) x[m][u] = ldv<T, V, UA>(src + sl[u]);
              }
#pragma unroll
              for (int u = 0; u < U; ++u)
#pragma unroll
                for (int i = 0; i < V; ++i) {
                  T a = wt[q][0] * x[0][u].v[i];
                  a = fma(wt[q][1], x[1][u].v[i], a);
                  a = fma(wt[q][2], x[2][u].v[i], a);
                  a = fma(wt[q][3], x[3][u].v[i], a);
                  y[q][u].v[i] = sign[u] * a;
                }
            }
            __builtin_amdgcn_sched_barrier(0);  // keep the next row's loads after this row's sum
          }
        } else {
          Pack<T, V> x[RB][4][U];
#pragma unroll
          for (int q = 0; q < RB; ++q)
#pragma unroll
            for (int m = 0; m < 4; ++m) {
              const T* src = f + (int64_t)c[q][m] * d.cs;
#pragma unroll
              for (int u = 0; u < U; ++u) x[q][m][u] = ldv<T, V, UA>(src + sl[u]);
            }
#pragma unroll
          for (int q = 0; q < RB; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
              for (int i = 0; i < V; ++i) {
                T a = wt[q][0] * x[q][0][u].v[i];
                a = fma(wt[q][1], x[q][1][u].v[i], a);
                a = fma(wt[q][2], x[q][2][u].v[i], a);
                a = fma(wt[q][3], x[q][3][u].v[i], a);
                y[q][u].v[i] = sign[u] * a;
              }
        }
      } else if ((KM & KM_GENERAL) && (kind == SEG_ELL || kind == SEG_CSR)) {
        // general rows (any width): entries in chunks of EC, each chunk's
        // columns and weights read together, then all its source loads, then
        // the sum in entry order (first product, then FMAs)
        constexpr int EC = 8;
#pragma unroll
        for (int q = 0; q < RB; ++q) {
#pragma unroll
          for (int u = 0; u < U; ++u)
#pragma unroll
            for (int i = 0; i < V; ++i) y[q][u].v[i] = T(0);
          if (r + q * rs >= re) continue;  // a batch slot past the group's rows
          int64_t e0, e1;
          const int32_t* cols;
          const T* vals;
          if (kind == SEG_ELL) {
            e0 = tl.tab + (int64_t)rr[q] * tl.width;
            e1 = e0 + tl.width;
            cols = d.ell_col;
            vals = static_cast<const T*>(d.ell_val);
          } else {
            e0 = d.csr_ptr[tl.tab + rr[q]];
            e1 = d.csr_ptr[tl.tab + rr[q] + 1];
            cols = d.csr_col;
            vals = static_cast<const T*>(d.csr_val);
          }
          bool first = true;
          for (int64_t eb = e0; eb < e1; eb += EC) {
            const int ne = (int)min<int64_t>(EC, e1 - eb);
            int32_t cc[EC];
            T wv[EC];
#pragma unroll
            for (int k = 0; k < EC; ++k) {
              cc[k] = -1;
              wv[k] = T(0);
              if (k < ne) {
                cc[k] = cols[eb + k];
                wv[k] = vals[eb + k];
              }
            }
            Pack<T, V> x[EC][U];
#pragma unroll
            for (int k = 0; k < EC; ++k)
              if (cc[k] >= 0) {
                const T* src = f + (int64_t)cc[k] * d.cs;
#pragma unroll
                for (int u = 0; u < U; ++u) x[k][u] = ldv<T, V, UA>(src + sl[u]);
              }
#pragma unroll
            for (int k = 0; k < EC; ++k)
              if (cc[k] >= 0) {
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                  for (int i = 0; i < V; ++i)
                    y[q][u].v[i] = first ? wv[k] * x[k][u].v[i] : fma(wv[k], x[k][u].v[i], y[q][u].v[i]);
                first = false;
              }
          }
#pragma unroll
          for (int u = 0; u < U; ++u)
#pragma unroll
            for (int i = 0; i < V; ++i) y[q][u].v[i] = sign[u] * y[q][u].v[i];
        }
      } else {  // zero rows, or b-only rows
#pragma unroll
        for (int q = 0; q < RB; ++q)
#pragma unroll
          for (int u = 0; u < U; ++u)
#pragma unroll
            for (int i = 0; i < V; ++i) y[q][u].v[i] = T(0);
      }
      if (with_b) {
#pragma unroll
        for (int q = 0; q < RB; ++q) {
          const T* bp = bt + (int64_t)rr[q] * tl.b_inner;
#pragma unroll
          for (int u = 0; u < U; ++u)
#pragma unroll
            for (int i = 0; i < V; ++i) {
              const T bb = tl.b_inner == 1 ? bp[0] : bp[l[u] + i];
              y[q][u].v[i] = kind == SEG_VEC ? bb : y[q][u].v[i] + bb;
            }
        }
      }
#pragma unroll
      for (int q = 0; q < RB; ++q)
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (r + q * rs < re && ok[u]) stv<T, V, NT, UA>(f + dst[q] * d.cs + l[u], y[q][u]);
    }
  }
}

// Zero rows of a row tile (point-major), written by extra workgroups of the
// wide-row launches when a plan's other rows are all zero rows without b, so
// that such a plan needs one launch.
template <typename T>
__device__ __forceinline__ void zero_row_tile(const PlanDesc& d, const RowTile& t) {
  T* __restrict__ f = static_cast<T*>(d.field);
  const int64_t inner = d.inner, n = (int64_t)t.nrows * inner;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
    const int64_t r = e / inner, l = e - r * inner;
    f[(int64_t)d.row_dst[t.row_begin + r] * d.cs + l] = T(0);
  }
}

// Lane k's value of a wavefront-uniform lane index k (v_readlane: no LDS).
__device__ __forceinline__ int rdl(int v, int k) { return __builtin_amdgcn_readlane(v, k); }
__device__ __forceinline__ float rdl(float v, int k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
__device__ __forceinline__ double rdl(double v, int k) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(b & 0xffffffffll), k);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
  return __longlong_as_double(((long long)hi << 32) | lo);
}

// Sliding-window rows (WinRun): one wavefront per (run, slice of 64 16-byte
// vectors).  Row r of a run reads cells r .. r + 3 of the run's window, so a
// run of R rows reads R + 3 cells.  Lane k < R first reads row k's
// destination and four weights; row r's values are then taken from lane r
// with v_readlane.  Every load of the run (its cells, 1 KiB per wavefront
// access) is issued before the first store: loads and stores share one
// in-order counter on this architecture, so a load issued after a store
// could not be waited for without also waiting for that store.  Rows are
// then summed and stored in order, each as soon as its last cell arrives.
// The sum is the general row path's (first product, then FMAs in entry
// order, then the component sign, then b), so both give the same bits.
// Workgroups past the window items write the plan's zero rows (ztiles), when
// those are all its other rows.
// Ordered form: the rows' destinations and weights, then the run's source
// rows, then the rows one after another.  The autotuner picks it where it is
// faster (at some run lengths it is, in FP32).
template <typename T, int V, bool NT, int RM>
__device__ __forceinline__ void win_ordered(const PlanDesc& d, const WinRun* __restrict__ runs, int nitems,
                                            int nslices, int zero_only, int b) {
  const int lane = (int)threadIdx.x & 63;
  const int item = b * 4 + ((int)threadIdx.x >> 6);
  if (item >= nitems) return;
  const int ri = item / nslices, slc = item - ri * nslices;
  const WinRun rn = runs[ri];
  T* __restrict__ f = static_cast<T*>(d.field);
  const int64_t nvec = d.inner / V;
  const int64_t vi = (int64_t)slc * 64 + lane;
  const bool ok = vi < nvec;
  const int64_t l = (ok ? vi : 0) * V;  // lanes past the row's end repeat vector 0 and store nothing
  T sign = T(1);
  const int64_t sl = rot_slot<T>(d, rn.rot, l, sign);
  const int R = rn.nrows;
  int my_dst = 0;
  T my_w[4] = {T(0), T(0), T(0), T(0)};
  if (lane < R) {
    my_dst = d.row_dst[rn.row_begin + lane];
    const T* wp = static_cast<const T*>(d.ell_val) + rn.tab + 4 * lane;
#pragma unroll
    for (int m = 0; m < 4; ++m) my_w[m] = wp[m];
  }
  if (zero_only) {
    Pack<T, V> z;
#pragma unroll
    for (int i = 0; i < V; ++i) z.v[i] = T(0);
#pragma unroll
    for (int r = 0; r < RM; ++r)
      if (r < R && ok) stv<T, V, NT>(f + (int64_t)rdl(my_dst, r) * d.cs + l, z);
    return;
  }
  const int64_t step = (int64_t)rn.dl * d.cs;
  const T* x0 = f + (int64_t)rn.src0 * d.cs + sl;
  Pack<T, V> x[RM + 3];
#pragma unroll
  for (int j = 0; j < RM + 3; ++j)
    if (j < R + 3) x[j] = ldv<T, V>(x0 + (int64_t)j * step);
  const T* __restrict__ bt = static_cast<const T*>(d.bval) + rn.brow;
#pragma unroll
  for (int r = 0; r < RM; ++r) {
    if (r < R) {
      const T c0 = rdl(my_w[0], r), c1 = rdl(my_w[1], r), c2 = rdl(my_w[2], r), c3 = rdl(my_w[3], r);
      Pack<T, V> y;
#pragma unroll
      for (int i = 0; i < V; ++i) {
        T a = c0 * x[r].v[i];
        a = fma(c1, x[r + 1].v[i], a);
        a = fma(c2, x[r + 2].v[i], a);
        a = fma(c3, x[r + 3].v[i], a);
        y.v[i] = sign * a;
      }
      if (rn.has_b) {
        const T* bp = bt + (int64_t)r * rn.b_inner;
#pragma unroll
        for (int i = 0; i < V; ++i) y.v[i] = y.v[i] + (rn.b_inner == 1 ? bp[0] : bp[l + i]);
      }
      if (ok) stv<T, V, NT>(f + (int64_t)rdl(my_dst, r) * d.cs + l, y);
    }
  }
}

// Pipelined form: scalar run descriptor; the rows' destinations and weights,
// the run's source rows and its b values in flight together; every store
// issued (see below) so that each row waits only for its own loads.
template <typename T, int V, bool NT, int RM, bool HB>
__device__ __forceinline__ void win_pipelined(const PlanDesc& d, const WinRun* __restrict__ runs, int nitems,
                                              int nslices, int zero_only, int b) {
  const int lane = (int)threadIdx.x & 63;
  // the wave's item is the same in every lane: the run descriptor comes
  // through scalar loads
  const int item = __builtin_amdgcn_readfirstlane(b * 4 + ((int)threadIdx.x >> 6));
  if (item >= nitems) return;
  const int ri = item / nslices, slc = item - ri * nslices;
  const WinRun rn = runs[ri];
  T* __restrict__ f = static_cast<T*>(d.field);
  const int64_t nvec = d.inner / V;
  const int64_t vi = (int64_t)slc * 64 + lane;
  const bool ok = vi < nvec;
  const int64_t l = (ok ? vi : 0) * V;  // lanes past the row's end repeat vector 0 and store nothing
  T sign = T(1);
  const int64_t sl = rot_slot<T>(d, rn.rot, l, sign);
  const int R = rn.nrows;
  // lane r holds row r's destination and weights (lanes past the run repeat
  // its last row; rows are read back with readlane)
  const int mr = min(lane, R - 1);
  if (zero_only) {
    const int my_dst = d.row_dst[rn.row_begin + mr];
    Pack<T, V> z;
#pragma unroll
    for (int i = 0; i < V; ++i) z.v[i] = T(0);
#pragma unroll
    for (int r = 0; r < RM; ++r)
      if (r < R && ok) stv<T, V, NT>(f + (int64_t)rdl(my_dst, r) * d.cs + l, z);
    return;
  }
  // the rows' destinations and weights, then the run's source rows, all in
  // flight together.  Every load is issued whatever R (spare slots re-read
  // the run's last source row) and every store too (through a buffer range
  // of its one destination row, with an out-of-range offset where nothing is
  // stored): loads and stores retire in issue order, and guarded ones would
  // make each row's store wait for the one before it.
  // the wave issues its loads at raised priority (s_setprio) and drops back
  // for the sums and stores.  Measured: C384 FP64 22.4 against 24.3 us at
  // the best run length (runs of 8-16 gain, runs of 4-6 lose, the autotuner
  // picks among them), FP32 11.2 against 11.8 us; priority 1 or 3, dropped
  // after the loads or before the stores, all give the same.  The same
  // bracket around the loads of the row, consumer, adjoint and wide-row
  // kernels gains nothing, and the 27-point march loses with it.
  __builtin_amdgcn_s_setprio(3);
  const int my_dst = d.row_dst[rn.row_begin + mr];
  T my_w[4];
  {
    const T* wp = static_cast<const T*>(d.ell_val) + rn.tab + 4 * mr;
#pragma unroll
    for (int m = 0; m < 4; ++m) my_w[m] = wp[m];
  }
  const int64_t step = (int64_t)rn.dl * d.cs;
  const T* x0 = f + (int64_t)rn.src0 * d.cs + sl;
  Pack<T, V> x[RM + 3];
#pragma unroll
  for (int j = 0; j < RM + 3; ++j) x[j] = ldv<T, V>(x0 + (int64_t)min(j, R + 2) * step);
  __builtin_amdgcn_s_setprio(0);
  auto row_value = [&](int r) {
    const T c0 = rdl(my_w[0], r), c1 = rdl(my_w[1], r), c2 = rdl(my_w[2], r), c3 = rdl(my_w[3], r);
    Pack<T, V> y;
#pragma unroll
    for (int i = 0; i < V; ++i) {
      T a = c0 * x[r].v[i];
      a = fma(c1, x[r + 1].v[i], a);
      a = fma(c2, x[r + 2].v[i], a);
      a = fma(c3, x[r + 3].v[i], a);
      y.v[i] = sign * a;
    }
    return y;
  };
  // b values of the run's rows, issued with the sources (a row past the run
  // re-reads the run's last one); one value per row is broadcast
  // (HB: the plan has runs with b; instances without it keep no registers for b)
  Pack<T, V> bv[HB ? RM : 1];
  if (HB && rn.has_b) {
    const T* __restrict__ bt = static_cast<const T*>(d.bval) + rn.brow;
#pragma unroll
    for (int r = 0; r < RM; ++r) {
      const T* bp = bt + (int64_t)min(r, R - 1) * rn.b_inner;
      if (rn.b_inner == 1) {
        const T b0 = bp[0];
#pragma unroll
        for (int i = 0; i < V; ++i) bv[r].v[i] = b0;
      } else {
        bv[r] = ldv<T, V>(bp + l);
      }
    }
  }
  const uint32_t off = ok ? (uint32_t)(l * (int64_t)sizeof(T)) : BUF_OOB;
  const int row_bytes = (int)(d.inner * (int64_t)sizeof(T));  // < 2 GiB (checked by the host)
#pragma unroll
  for (int r = 0; r < RM; ++r) {
    Pack<T, V> y = row_value(r);
    if constexpr (HB) {
      if (rn.has_b) {
#pragma unroll
        for (int i = 0; i < V; ++i) y.v[i] = y.v[i] + bv[r].v[i];
      }
    }
    const __amdgpu_buffer_rsrc_t dr = __builtin_amdgcn_make_buffer_rsrc(
        f + (int64_t)rdl(my_dst, min(r, R - 1)) * d.cs, 0, row_bytes, BUF_RSRC_WORD3);
    stv_buf<T, V, NT>(y, dr, r < R ? off : BUF_OOB);
  }
}

template <typename T, int V, bool NT, int RM, bool ORD, bool HB>
__global__ __launch_bounds__(256) void k_apply_win(PlanDesc d, const WinRun* __restrict__ runs, int nitems,
                                                   int nslices, int zero_only, const RowTile* __restrict__ ztiles,
                                                   int nz) {
  const int nwin = (nitems + 3) >> 2;
  if ((int)blockIdx.x >= nwin) {
    for (int t = (int)blockIdx.x - nwin; t < nz; t += (int)gridDim.x - nwin) zero_row_tile<T>(d, ztiles[t]);
    return;
  }
  // workgroups are dealt to the 8 XCDs round-robin: give each XCD a
  // contiguous range of runs (neighbouring runs share three cells)
  int b = (int)blockIdx.x;
  {
    const int q = nwin >> 3, rem = nwin & 7, x = b & 7, jx = b >> 3;
    b = x * q + min(x, rem) + jx;
  }
  if constexpr (ORD)
    win_ordered<T, V, NT, RM>(d, runs, nitems, nslices, zero_only, b);
  else
    win_pipelined<T, V, NT, RM, HB>(d, runs, nitems, nslices, zero_only, b);
}

// One entry of a wide tile: its weight and the LDS offset (in values) of its
// source cell's staged slice, read with one LDS instruction.
template <typename T>
struct alignas(2 * sizeof(T)) WideEnt {
  T w;
  int32_t slot;
};

template <typename T>
__device__ __forceinline__ void ld_ent(const WideEnt<T>* p, T& w, int& slot) {
  if constexpr (sizeof(T) == 8) {
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
    const u4 v = *reinterpret_cast<const u4*>(p);
    w = __builtin_bit_cast(double, ((uint64_t)v[1] << 32) | v[0]);
    slot = (int)v[2];
  } else {
    typedef uint32_t u2 __attribute__((ext_vector_type(2)));
    const u2 v = *reinterpret_cast<const u2*>(p);
    w = __builtin_bit_cast(float, v[0]);
    slot = (int)v[1];
  }
}

// Wide rows (WideTile).  A workgroup takes one tile and a run of spw
// consecutive slices of SB bytes of inner values.  The tile's entries
// and row starts go to LDS once; then, per slice, the tile's distinct source
// cells are staged in LDS (the slots this slice's outputs read, through the
// component rotation) and a group of lanes per row sums the row's entries
// from LDS in entry order, EC entries per step with every LDS read of the
// step issued first.  The sum starts from -0.0 and takes only FMAs, which
// gives the same bits as a first product followed by FMAs (the general row
// path); the row's last partial step re-reads its last entry for the
// missing ones and drops them by a select, so no step branches per entry.
// The next slice's staging loads are in flight while the current slice is
// summed.  LDS holds ucap cells of the slice, then ecap entries, then the
// row starts.  zero_only writes +0 to the tile's rows (the adjoint's ghost
// reset).
template <typename T, int V, int SB, bool NT>
__global__ __launch_bounds__(256) void k_apply_wide(PlanDesc d, const WideTile* __restrict__ tiles,
                                                    const int32_t* __restrict__ ucell,
                                                    const int32_t* __restrict__ wrow,
                                                    const int32_t* __restrict__ wrp,
                                                    const WideEnt<T>* __restrict__ went, int ucap, int ecap,
                                                    int nslices, int spw, int zero_only,
                                                    const RowTile* __restrict__ ztiles, int nwide) {
  extern __shared__ __align__(16) unsigned char wide_smem[];
  constexpr int S = SB / (int)sizeof(T);              // values per cell and slice
  constexpr int LPR = S / V;                          // lanes per row
  constexpr int NGRP = 256 / LPR;                     // row groups (launched with 256 threads)
  constexpr int RPG = (WIDE_ROWS + NGRP - 1) / NGRP;  // rows per group
  constexpr int NIT = (WIDE_UCAP * LPR + 255) / 256;  // staging items per thread
  constexpr int NE = (WIDE_ECAP + 255) / 256;
  constexpr int EC = 4;                               // entries per step
  T* lds = reinterpret_cast<T*>(wide_smem);                                            // ucap x S values
  WideEnt<T>* le = reinterpret_cast<WideEnt<T>*>(wide_smem + (size_t)ucap * SB);  // ecap entries
  int32_t* lp = reinterpret_cast<int32_t*>(le + ecap);                                 // WIDE_ROWS + 1 row starts
  if ((int)blockIdx.x >= nwide) {  // a zero-row tile (no barrier is reached)
    zero_row_tile<T>(d, ztiles[blockIdx.x - nwide]);
    return;
  }
  // workgroups are dealt to the 8 XCDs round-robin: give each XCD a
  // contiguous range of (tile, slice group) items, so that neighbouring
  // tiles, which share source cells, meet in one L2
  int b = (int)blockIdx.x;
  {
    const int q = nwide >> 3, rem = nwide & 7, x = b & 7, jx = b >> 3;
    b = x * q + min(x, rem) + jx;
  }
  const int runs = (nslices + spw - 1) / spw;
  const WideTile tl = tiles[b / runs];
  const int s0 = (b % runs) * spw;
  const int s1 = min(nslices, s0 + spw);
  T* __restrict__ f = static_cast<T*>(d.field);
  typedef T vt __attribute__((ext_vector_type(V)));
  const int lane = threadIdx.x % LPR, grp = threadIdx.x / LPR;
  int32_t ridx[RPG];
  int64_t dst[RPG];
#pragma unroll
  for (int q = 0; q < RPG; ++q) {
    const int r = grp + q * NGRP;
    ridx[q] = r < tl.nrows ? wrow[tl.r0 + r] : 0;
  }
#pragma unroll
  for (int q = 0; q < RPG; ++q) dst[q] = grp + q * NGRP < tl.nrows ? d.row_dst[tl.row_base + ridx[q]] : 0;
  if (zero_only) {
    for (int s = s0; s < s1; ++s) {
      const int64_t l = (int64_t)s * S + lane * V;
      if (l >= d.inner) continue;
      Pack<T, V> z;
#pragma unroll
      for (int i = 0; i < V; ++i) z.v[i] = T(0);
#pragma unroll
      for (int q = 0; q < RPG; ++q)
        if (grp + q * NGRP < tl.nrows) stv<T, V, NT>(f + dst[q] * d.cs + l, z);
    }
    return;
  }
  // Per staging item (the same for every slice): the source cell's address
  // and the item's slot offset; per slice only 32-bit slot arithmetic (inner
  // extents of wide plans stay below 2^30) and, for rotated tiles, the
  // component rotation remain.  An item's LDS offset is (thread + 256 k) * V.
  const int inner = (int)d.inner, vlo = (int)d.vec_lo, vst = (int)d.vec_stride, vlen = (int)d.vec_len;
  const bool rotates = tl.rot != 0 && vlen != 0;
  auto rslot = [&](int l, T& sign) -> int {  // rot_slot in 32-bit
    sign = T(1);
    if (!rotates) return l;
    int off = l - vlo, a;
    if (off >= 0 && off < vlen) {
      a = 0;
    } else if (off >= vst && off < vst + vlen) {
      a = 1;
      off -= vst;
    } else {
      return l;
    }
    if (tl.rot & (2 << a)) sign = T(-1);
    return vlo + ((tl.rot & 1) ? 1 - a : a) * vst + off;
  };
  const T* sp[NIT];
  uint32_t live = 0;  // bit k: item k is one of the tile's cells
#pragma unroll
  for (int k = 0; k < NIT; ++k) {
    const int u = (threadIdx.x + k * 256) / LPR;
    sp[k] = f;
    if (u < tl.nu) {
      sp[k] = f + (int64_t)ucell[tl.first_u + u] * d.cs;
      live |= 1u << k;
    }
  }
  Pack<T, V> g[NIT];
  auto issue = [&](int s) {
    const int l0 = s * S;
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int lv = l0 + ((threadIdx.x + k * 256) % LPR) * V;
      if ((live >> k & 1u) && lv < inner) {
        T sign;
        g[k] = ldv<T, V>(sp[k] + rslot(lv, sign));
      }
    }
  };
  issue(s0);
  {
    // entries move as plain vectors (a struct copy would go through scratch)
    typedef uint32_t eu __attribute__((ext_vector_type(sizeof(WideEnt<T>) / 4)));
    const eu* __restrict__ gsrc = reinterpret_cast<const eu*>(went + tl.e0);
    eu* ldst = reinterpret_cast<eu*>(le);
    eu ev[NE];
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int e = threadIdx.x + k * 256;
      if (e < tl.ne) ev[k] = gsrc[e];
    }
    int32_t rp = 0;
    if ((int)threadIdx.x <= tl.nrows) rp = wrp[tl.rp0 + threadIdx.x];
#pragma unroll
    for (int k = 0; k < NE; ++k) {
      const int e = threadIdx.x + k * 256;
      if (e < tl.ne) ldst[e] = ev[k];
    }
    if ((int)threadIdx.x <= tl.nrows) lp[threadIdx.x] = rp;
  }
  T* dp[RPG];
#pragma unroll
  for (int q = 0; q < RPG; ++q) dp[q] = f + dst[q] * d.cs;
  const T* __restrict__ bt = static_cast<const T*>(d.bval) + tl.brow;
  for (int s = s0; s < s1; ++s) {
    const int l0 = s * S;
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int e = threadIdx.x + k * 256;
      if ((live >> k & 1u) && l0 + (e % LPR) * V < inner) {
        vt w;
#pragma unroll
        for (int i = 0; i < V; ++i) w[i] = g[k].v[i];
        *reinterpret_cast<vt*>(&lds[e * V]) = w;
      }
    }
    __syncthreads();
    if (s + 1 < s1) issue(s + 1);
    const int l = l0 + lane * V;
    if (l < inner) {
      T sign;
      (void)rslot(l, sign);
      const T* __restrict__ xl = lds + lane * V;
#pragma unroll
      for (int q = 0; q < RPG; ++q) {
        const int r = grp + q * NGRP;
        if (r >= tl.nrows) break;
        const int e0 = lp[r], e1 = lp[r + 1];
        vt y;
#pragma unroll
        for (int i = 0; i < V; ++i) y[i] = e1 > e0 ? T(-0.0) : T(0);
        int c = e0;
        for (; c + EC <= e1; c += EC) {
          T w[EC];
          int o[EC];
#pragma unroll
          for (int m = 0; m < EC; ++m) ld_ent<T>(le + c + m, w[m], o[m]);
          vt x[EC];
#pragma unroll
          for (int m = 0; m < EC; ++m) x[m] = *reinterpret_cast<const vt*>(xl + o[m]);
#pragma unroll
          for (int m = 0; m < EC; ++m)
#pragma unroll
            for (int i = 0; i < V; ++i) y[i] = fma(w[m], x[m][i], y[i]);
        }
        if (c < e1) {  // the last 1..EC-1 entries: clamped reads, dead steps dropped by a select
          T w[EC - 1];
          int o[EC - 1];
#pragma unroll
          for (int m = 0; m < EC - 1; ++m) ld_ent<T>(le + min(c + m, e1 - 1), w[m], o[m]);
          vt x[EC - 1];
#pragma unroll
          for (int m = 0; m < EC - 1; ++m) x[m] = *reinterpret_cast<const vt*>(xl + o[m]);
#pragma unroll
          for (int m = 0; m < EC - 1; ++m) {
            const bool lv = c + m < e1;
#pragma unroll
            for (int i = 0; i < V; ++i) y[i] = lv ? fma(w[m], x[m][i], y[i]) : y[i];
          }
        }
        Pack<T, V> o;
#pragma unroll
        for (int i = 0; i < V; ++i) o.v[i] = sign * y[i];
        if (tl.has_b) {
          const T* bp = bt + (int64_t)ridx[q] * tl.b_inner;
#pragma unroll
          for (int i = 0; i < V; ++i) o.v[i] += tl.b_inner == 1 ? bp[0] : bp[l + i];
        }
        stv<T, V, NT>(dp[q] + l, o);
      }
    }
    __syncthreads();
  }
}

// Narrow wide rows (NarrowTile): rows of >= WIDE_NNZ entries and fewer than
// NARROW_ROW_BYTES (a few inner values).  A group of NARROW_LANES lanes takes
// one row: lane j sums entries j, j + NARROW_LANES, ... of the row for every
// source slot (starting from -0.0, the additive identity, with FMAs; two
// entries' loads in flight at a time), the partial sums are added across
// the group by an xor butterfly (every lane ends with the same bits), and
// lane l < inner writes output slot l through the component rotation.  The
// order of the sum differs from the general row path, the result is
// deterministic.  zero_only writes +0 to the tile's rows.
template <typename T>
__global__ __launch_bounds__(256) void k_apply_narrow(PlanDesc d, const NarrowTile* __restrict__ tiles,
                                                      int zero_only, const RowTile* __restrict__ ztiles,
                                                      int nnarrow) {
  constexpr int G = NARROW_LANES, IM = NARROW_ROW_BYTES / (int)sizeof(T);
  if ((int)blockIdx.x >= nnarrow) {  // a zero-row tile
    zero_row_tile<T>(d, ztiles[blockIdx.x - nnarrow]);
    return;
  }
  const NarrowTile tl = tiles[blockIdx.x];
  const int j = threadIdx.x % G, rr = threadIdx.x / G;
  const bool live = rr < tl.nrows;  // every lane takes part in the butterfly
  const int inner = (int)d.inner;
  T* __restrict__ f = static_cast<T*>(d.field);
  const T* __restrict__ vals = static_cast<const T*>(d.csr_val);
  int64_t e0 = 0, e1 = 0, dst = 0;
  if (live) {
    e0 = d.csr_ptr[tl.tab + rr];
    e1 = d.csr_ptr[tl.tab + rr + 1];
    dst = d.row_dst[tl.row_begin + rr];
  }
  T p[IM];
#pragma unroll
  for (int l = 0; l < IM; ++l) p[l] = T(-0.0);
  if (!zero_only) {
    for (int64_t e = e0 + j; e < e1; e += 2 * G) {
      const bool two = e + G < e1;
      const int64_t c0 = d.csr_col[e], c1 = two ? d.csr_col[e + G] : c0;
      const T w0 = vals[e], w1 = two ? vals[e + G] : T(0);
      T x0[IM], x1[IM];
#pragma unroll
      for (int l = 0; l < IM; ++l)
        if (l < inner) {
          x0[l] = f[c0 * d.cs + l];
          x1[l] = f[c1 * d.cs + l];
        }
#pragma unroll
      for (int l = 0; l < IM; ++l)
        if (l < inner) {
          p[l] = fma(w0, x0[l], p[l]);
          if (two) p[l] = fma(w1, x1[l], p[l]);
        }
    }
#pragma unroll
    for (int off = G / 2; off >= 1; off /= 2)
#pragma unroll
      for (int l = 0; l < IM; ++l)
        if (l < inner) p[l] += __shfl_xor(p[l], off, G);
  }
  if (!live || j >= inner) return;
  T out = T(0);
  if (!zero_only) {
    T sign;
    const int src = (int)rot_slot<T>(d, tl.rot, j, sign);
    T v = p[0];
#pragma unroll
    for (int m = 1; m < IM; ++m)
      if (m == src) v = p[m];
    out = sign * (e1 > e0 ? v : T(0));
    if (tl.has_b) {
      const T* bp = static_cast<const T*>(d.bval) + tl.brow + (int64_t)rr * tl.b_inner;
      out += tl.b_inner == 1 ? bp[0] : bp[j];
    }
  }
  f[dst * d.cs + j] = out;
}

// Data rows (block-edge averaging).  Every row of an apply reads the input
// field, so data rows are first computed into scratch by extra workgroups of
// the ghost-row launch (they only read data cells and write scratch), and
// written by k_data_scatter after it.  A row's entries are read 4 at a time,
// all loads issued before the ordered sum.  A row group of lpr lanes takes one
// row; entries are summed in table order (first product, then FMAs), one
// thread per value.
struct DataDesc {
  const int64_t* ptr;
  const int32_t* col;
  const void* val;
  void* scratch;
  int32_t nrows;
  int32_t grid;  // workgroups of the launch that gather data rows (0: none)
};

template <typename T, int V>
__device__ __forceinline__ void data_gather_rows(const PlanDesc& d, const DataDesc& dd, int wg, int nwg) {
  const int lpr = 1 << d.lpr_shift;
  const int ngroups = (int)blockDim.x >> d.lpr_shift;
  const int lane = threadIdx.x & (lpr - 1), grp = threadIdx.x >> d.lpr_shift;
  const T* __restrict__ f = static_cast<const T*>(d.field);
  const T* __restrict__ val = static_cast<const T*>(dd.val);
  T* __restrict__ scratch = static_cast<T*>(dd.scratch);
  const int64_t nvec = d.inner / V;
  for (int r = wg * ngroups + grp; r < dd.nrows; r += nwg * ngroups) {
    const int64_t e0 = dd.ptr[r], e1 = dd.ptr[r + 1];
    for (int64_t v = lane; v < nvec; v += lpr) {
      const int64_t l = v * V;
      Pack<T, V> acc;
#pragma unroll
      for (int i = 0; i < V; ++i) acc.v[i] = T(0);
      bool first = true;
      for (int64_t eb = e0; eb < e1; eb += 4) {  // 4 entries' loads in flight, then the ordered sum
        const int ne = (int)min<int64_t>(4, e1 - eb);
        T w[4];
        Pack<T, V> x[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (j < ne) {
            w[j] = val[eb + j];
            x[j] = ldv<T, V>(f + (int64_t)dd.col[eb + j] * d.cs + l);
          }
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (j < ne) {
#pragma unroll
            for (int i = 0; i < V; ++i) acc.v[i] = first ? w[j] * x[j].v[i] : fma(w[j], x[j].v[i], acc.v[i]);
            first = false;
          }
      }
      stv<T, V, false>(scratch + (int64_t)r * d.inner + l, acc);
    }
  }
}

template <typename T, int V, int U, bool NT, int RB, int KM>
__global__ __launch_bounds__(256) void k_apply_rows(PlanDesc d, const RowTile* __restrict__ tiles, int ntiles,
                                                    int zero_only, DataDesc dd) {
  // the first dd.grid workgroups gather data rows (dispatched first, they
  // overlap the ghost-row tiles)
  if ((int)blockIdx.x < dd.grid) {
    data_gather_rows<T, V>(d, dd, (int)blockIdx.x, dd.grid);
    return;
  }
  const int main = (int)gridDim.x - dd.grid;
  for (int t = (int)blockIdx.x - dd.grid; t < ntiles; t += main) {
    const RowTile tl = tiles[t];
    rt_tile<T, V, U, NT, RB, KM>(d, tl, zero_only != 0);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_apply_pm(PlanDesc d, const DevTile* __restrict__ tiles, int ntiles,
                                                   int zero_only) {
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const DevTile tl = tiles[t];
    const DevSeg s = d.segs[tl.seg];
    run_tile_pm<T>(d, s, tl.row0, tl.nrows, zero_only != 0, threadIdx.x, blockDim.x);
  }
}

// Batch tiles of different plans: (vec, unroll) chosen per tile at run time.
template <typename T, bool NT, int KM>
__device__ __forceinline__ void rt_tile_any(const PlanDesc& d, const RowTile& tl) {
  if (d.ua) {
    rt_tile<T, (sizeof(T) == 4 ? 4 : 2), 1, NT, 4, KM | KM_UNAL>(d, tl, false);
    return;
  }
  if (sizeof(T) == 4) {
    if (d.vec == 4)
      rt_tile<T, (sizeof(T) == 4 ? 4 : 2), 1, NT, 4, KM>(d, tl, false);
    else if (d.vec == 2)  // unrolled rows take batches of 2 (registers of the whole batch kernel)
      d.unroll >= 2 ? rt_tile<T, 2, 2, NT, 2, KM>(d, tl, false) : rt_tile<T, 2, 1, NT, 4, KM>(d, tl, false);
    else if (d.unroll >= 4)
      rt_tile<T, 1, 4, NT, 2, KM>(d, tl, false);
    else
      d.unroll >= 2 ? rt_tile<T, 1, 2, NT, 2, KM>(d, tl, false) : rt_tile<T, 1, 1, NT, 4, KM>(d, tl, false);
  } else {
    if (d.vec >= 2)
      rt_tile<T, 2, 1, NT, 4, KM>(d, tl, false);
    else
      d.unroll >= 2 ? rt_tile<T, 1, 2, NT, 2, KM>(d, tl, false) : rt_tile<T, 1, 1, NT, 4, KM>(d, tl, false);
  }
}

template <typename T, int KM>
__global__ __launch_bounds__(256) void k_batch(const PlanDesc* __restrict__ descs, const RowTile* __restrict__ tiles,
                                               int ntiles) {
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const RowTile tl = tiles[t];
    const PlanDesc d = descs[tl.pad_];
    if (d.nt)
      rt_tile_any<T, true, KM>(d, tl);
    else
      rt_tile_any<T, false, KM>(d, tl);
  }
}

// Adjoint gather: for each source cell, in ascending ghost order,
//   xbar[src, l] += sum_e w_e * sign_e * ybar[ghost_e, rot_e(l)]
// One thread sums one value, so the result does not depend on scheduling.
// A source's entries come from the fixed-width table (no pointer to chase:
// the source index, its count and its entries are read together, then all
// its ybar loads are issued, then the ordered sum); sources with more than aw
// entries walk the CSR form in chunks of EB.
constexpr int EB = 8;

template <typename T, int V, bool ROWFAST, bool NT>
__global__ __launch_bounds__(256) void k_adjoint(PlanDesc d, AdjDesc a, const AdjTile* __restrict__ tiles,
                                                  int ntiles) {
  const int lpr = 1 << d.lpr_shift;
  const int ngroups = (int)blockDim.x >> d.lpr_shift;
  int lane, grp;
  if (ROWFAST) {
    grp = threadIdx.x % ngroups;
    lane = threadIdx.x / ngroups;
  } else {
    lane = threadIdx.x & (lpr - 1);
    grp = threadIdx.x >> d.lpr_shift;
  }
  const int64_t nvec = d.inner / V;
  T* __restrict__ f = static_cast<T*>(d.field);
  const T* __restrict__ W = static_cast<const T*>(a.w);
  const T* __restrict__ FW = static_cast<const T*>(a.fw);
  const int aw = a.aw;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const AdjTile tl = tiles[t];
    int rb, re, rs;
    if (!ROWFAST && d.chunked) {
      const int ch = (tl.count + ngroups - 1) / ngroups;
      rb = grp * ch;
      re = min(tl.count, rb + ch);
      rs = 1;
    } else {
      rb = grp;
      re = tl.count;
      rs = ngroups;
    }
    for (int r = rb; r < re; r += rs) {
      const int64_t k = tl.first + r;
      const int64_t cell = a.src[k];
      const int cnt = a.cnt[k];
      int32_t fg[ADJ_MAXW];
      T fwt[ADJ_MAXW];
      int fr[ADJ_MAXW];
#pragma unroll
      for (int m = 0; m < ADJ_MAXW; ++m) {
        fg[m] = 0;
        fwt[m] = T(0);
        fr[m] = 0;
        if (m < aw) {
          fg[m] = a.fg[k * aw + m];
          fwt[m] = FW[k * aw + m];
          fr[m] = a.frot[k * aw + m];
        }
      }
      for (int64_t v = lane; v < nvec; v += lpr) {
        const int64_t l = v * V;
        T* px = f + cell * d.cs + l * d.ls;
        Pack<T, V> x;
        if (ROWFAST) {
#pragma unroll
          for (int i = 0; i < V; ++i) x.v[i] = px[i * d.ls];
        } else {
          x = ldv<T, V>(px);
        }
        Pack<T, V> acc;
        if (cnt <= aw) {
          Pack<T, V> g[ADJ_MAXW];
          T wt[ADJ_MAXW];
#pragma unroll
          for (int m = 0; m < ADJ_MAXW; ++m) {
            if (m < cnt) {
              T sign;
              const int64_t sl = rot_slot<T>(d, fr[m], l, sign);
              wt[m] = fwt[m] * sign;
              g[m] = ldv<T, V>(f + (int64_t)fg[m] * d.cs + sl * d.ls);
            }
          }
#pragma unroll
          for (int i = 0; i < V; ++i) acc.v[i] = wt[0] * g[0].v[i];
#pragma unroll
          for (int m = 1; m < ADJ_MAXW; ++m)
            if (m < cnt) {
#pragma unroll
              for (int i = 0; i < V; ++i) acc.v[i] = fma(wt[m], g[m].v[i], acc.v[i]);
            }
        } else {
          const int64_t e0 = a.ptr[k], e1 = a.ptr[k + 1];
#pragma unroll
          for (int i = 0; i < V; ++i) acc.v[i] = T(0);
          bool first = true;
          for (int64_t eb = e0; eb < e1; eb += EB) {
            const int ne = (int)min<int64_t>(EB, e1 - eb);
            int64_t off[EB];
            T wt[EB];
#pragma unroll
            for (int j = 0; j < EB; ++j) {
              const int64_t e = eb + min(j, ne - 1);
              T sign;
              const int64_t sl = rot_slot<T>(d, a.rot[e], l, sign);
              wt[j] = W[e] * sign;
              off[j] = a.ghost[e] * d.cs + sl * d.ls;
            }
            Pack<T, V> g[EB];
#pragma unroll
            for (int j = 0; j < EB; ++j)
              if (j < ne) g[j] = ldv<T, V>(f + off[j]);
#pragma unroll
            for (int j = 0; j < EB; ++j) {
              if (j >= ne) break;
#pragma unroll
              for (int i = 0; i < V; ++i) acc.v[i] = first ? wt[j] * g[j].v[i] : fma(wt[j], g[j].v[i], acc.v[i]);
              first = false;
            }
          }
        }
#pragma unroll
        for (int i = 0; i < V; ++i) x.v[i] = x.v[i] + acc.v[i];
        if (ROWFAST) {
#pragma unroll
          for (int i = 0; i < V; ++i) px[i * d.ls] = x.v[i];
        } else {
          stv<T, V, NT>(px, x);
        }
      }
    }
  }
}

// Data rows in closed components (block-edge averaging: a component is one
// co-located set): a row group reads all of a component's columns into
// registers, then computes and writes its rows, so no scratch is needed; it
// runs after the ghost rows, which read the input values.  Sums in table
// order, as k_data_scatter's rows.
template <typename T, int V, bool NT>
__global__ __launch_bounds__(256) void k_data_components(PlanDesc d, const DataComp* __restrict__ comps,
                                                         const int32_t* __restrict__ row_dst,
                                                         const int32_t* __restrict__ row_ent,
                                                         const int32_t* __restrict__ row_n,
                                                         const int32_t* __restrict__ slot, const T* __restrict__ w,
                                                         int ncomp) {
  const int lpr = 1 << d.lpr_shift;
  const int ngroups = (int)blockDim.x >> d.lpr_shift;
  const int lane = threadIdx.x & (lpr - 1), grp = threadIdx.x >> d.lpr_shift;
  T* __restrict__ f = static_cast<T*>(d.field);
  const int64_t nvec = d.inner / V;
  for (int c = blockIdx.x * ngroups + grp; c < ncomp; c += gridDim.x * ngroups) {
    const DataComp cp = comps[c];
    for (int64_t v = lane; v < nvec; v += lpr) {
      const int64_t l = v * V;
      Pack<T, V> x[DC_MAX];
#pragma unroll
      for (int m = 0; m < DC_MAX; ++m)
        if (m < cp.ncol) x[m] = ldv<T, V>(f + (int64_t)cp.col[m] * d.cs + l);
      for (int k = 0; k < cp.nrow; ++k) {
        const int r = cp.first_row + k;
        const int e0 = row_ent[r], ne = row_n[r];
        Pack<T, V> acc;
#pragma unroll
        for (int i = 0; i < V; ++i) acc.v[i] = T(0);
#pragma unroll
        for (int j = 0; j < DC_MAX; ++j) {
          if (j >= ne) break;
          const int sj = slot[e0 + j];
          const T wj = w[e0 + j];
          Pack<T, V> xs = x[0];
#pragma unroll
          for (int m = 1; m < DC_MAX; ++m)
            if (m == sj) xs = x[m];
#pragma unroll
          for (int i = 0; i < V; ++i) acc.v[i] = j == 0 ? wj * xs.v[i] : fma(wj, xs.v[i], acc.v[i]);
        }
        stv<T, V, NT>(f + (int64_t)row_dst[r] * d.cs + l, acc);
      }
    }
  }
}

template <typename T, int V>
__global__ __launch_bounds__(256) void k_data_scatter(PlanDesc d, const int32_t* __restrict__ cell,
                                                      const T* __restrict__ scratch, int nrows) {
  const int lpr = 1 << d.lpr_shift;
  const int ngroups = (int)blockDim.x >> d.lpr_shift;
  const int lane = threadIdx.x & (lpr - 1), grp = threadIdx.x >> d.lpr_shift;
  T* __restrict__ f = static_cast<T*>(d.field);
  const int64_t nvec = d.inner / V;
  for (int r = blockIdx.x * ngroups + grp; r < nrows; r += gridDim.x * ngroups) {
    const int64_t dst = cell[r];
    for (int64_t v = lane; v < nvec; v += lpr) {
      const int64_t l = v * V;
      const Pack<T, V> x = ldv<T, V>(scratch + (int64_t)r * d.inner + l);
      if (d.nt)
        stv<T, V, true>(f + dst * d.cs + l, x);
      else
        stv<T, V, false>(f + dst * d.cs + l, x);
    }
  }
}

// LDS-staged adjoint (point-major).  Per tile: the distinct ghost rows its
// sources read are loaded into LDS once; each row is then retired (zeroed by
// this tile if it is the row's only reader tile, or the last one to
// decrement the row's reader counter, which it then restores); then each
// source sums its entries from LDS in ascending ghost order, exactly as the
// CSR-walking kernel does, so both give the same bits.  Workgroups past the
// tiles zero the covered ghost rows that no source reads.
struct AdjLdsDesc {
  const AdjLdsTile* tiles;
  const int32_t* ucell;
  const int32_t* uctr;
  const int32_t* ctrinit;
  int32_t* ctr;
  const uint16_t* slot;
  const int32_t* zero;
  int32_t ntiles;
  int32_t nzero;
};

template <typename T, int V, bool NT>
__global__ __launch_bounds__(256) void k_adjoint_lds(PlanDesc d, AdjDesc a, AdjLdsDesc q) {
  extern __shared__ __align__(16) unsigned char adj_smem[];
  T* rows = reinterpret_cast<T*>(adj_smem);
  __shared__ int zflag[ADJ_LDS_ROWS];
  typedef T vt __attribute__((ext_vector_type(V)));
  T* __restrict__ f = static_cast<T*>(d.field);
  const int64_t inner = d.inner;
  const int nvec = (int)(inner / V);
  Pack<T, V> zero;
#pragma unroll
  for (int i = 0; i < V; ++i) zero.v[i] = T(0);
  if ((int)blockIdx.x >= q.ntiles) {
    const int r0 = ((int)blockIdx.x - q.ntiles) * ADJ_ZERO_ROWS;
    const int nr = min(ADJ_ZERO_ROWS, q.nzero - r0);
    for (int e = threadIdx.x; e < nr * nvec; e += blockDim.x) {
      const int r = e / nvec, v = e - r * nvec;
      stv<T, V, NT>(f + (int64_t)q.zero[r0 + r] * d.cs + (int64_t)v * V, zero);
    }
    return;
  }
  // workgroups are dealt to the 8 XCDs round-robin: give each XCD a
  // contiguous range of tiles (neighbouring tiles read shared ghost rows)
  int bt = (int)blockIdx.x;
  {
    const int nq = q.ntiles >> 3, rem = q.ntiles & 7, x = bt & 7, jx = bt >> 3;
    bt = x * nq + min(x, rem) + jx;
  }
  const AdjLdsTile tl = q.tiles[bt];
  const int nu = tl.nu;
  // staging: SG vector loads of ghost rows in flight per thread, then their
  // LDS stores (row u of the tile at u * inner)
  constexpr int SG = 4;
  const int nstage = nu * nvec, bd = (int)blockDim.x;
  for (int e0 = threadIdx.x; e0 < nstage; e0 += SG * bd) {
    Pack<T, V> g[SG];
#pragma unroll
    for (int j = 0; j < SG; ++j) {
      const int e = e0 + j * bd;
      if (e < nstage) {
        const int u = e / nvec, v = e - u * nvec;
        g[j] = ldv<T, V>(f + (int64_t)q.ucell[tl.first_u + u] * d.cs + (int64_t)v * V);
      }
    }
#pragma unroll
    for (int j = 0; j < SG; ++j) {
      const int e = e0 + j * bd;
      if (e < nstage) {
        vt w;
#pragma unroll
        for (int i = 0; i < V; ++i) w[i] = g[j].v[i];
        *reinterpret_cast<vt*>(&rows[(int64_t)e * V]) = w;  // = u * inner + v * V
      }
    }
  }
  __syncthreads();  // every load of this tile's ghost rows has returned
  for (int u = threadIdx.x; u < nu; u += blockDim.x) {
    const int c = q.uctr[tl.first_u + u];
    int z = 1;
    if (c >= 0) {
      z = atomicSub(&q.ctr[c], 1) == 1 ? 1 : 0;
      if (z) atomicExch(&q.ctr[c], q.ctrinit[c]);
    }
    zflag[u] = z;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nu * nvec; e += blockDim.x) {
    const int u = e / nvec, v = e - u * nvec;
    if (zflag[u]) stv<T, V, NT>(f + (int64_t)q.ucell[tl.first_u + u] * d.cs + (int64_t)v * V, zero);
  }
  const int lpr = 1 << d.lpr_shift;
  const int ngroups = (int)blockDim.x >> d.lpr_shift;
  const int lane = threadIdx.x & (lpr - 1), grp = threadIdx.x >> d.lpr_shift;
  const T* __restrict__ FW = static_cast<const T*>(a.fw);
  const int aw = a.aw;
  for (int r = grp; r < tl.nsrc; r += ngroups) {
    const int64_t k = tl.first_src + r;
    const int64_t cell = a.src[k];
    const int cnt = a.cnt[k];
    int sl_[ADJ_MAXW];
    T fwt[ADJ_MAXW];
    int fr[ADJ_MAXW];
#pragma unroll
    for (int m = 0; m < ADJ_MAXW; ++m) {
      sl_[m] = 0;
      fwt[m] = T(0);
      fr[m] = 0;
      if (m < aw) {
        sl_[m] = q.slot[k * aw + m];
        fwt[m] = FW[k * aw + m];
        fr[m] = a.frot[k * aw + m];
      }
    }
    for (int v = lane; v < nvec; v += lpr) {
      const int64_t l = (int64_t)v * V;
      T* px = f + cell * d.cs + l;
      Pack<T, V> x = ldv<T, V>(px);
      Pack<T, V> acc;
#pragma unroll
      for (int m = 0; m < ADJ_MAXW; ++m) {
        if (m < cnt) {
          T sign;
          const int64_t sl = rot_slot<T>(d, fr[m], l, sign);
          const T wt = fwt[m] * sign;
          const vt g = *reinterpret_cast<const vt*>(&rows[(int64_t)sl_[m] * inner + sl]);
#pragma unroll
          for (int i = 0; i < V; ++i) acc.v[i] = m == 0 ? wt * g[i] : fma(wt, g[i], acc.v[i]);
        }
      }
#pragma unroll
      for (int i = 0; i < V; ++i) x.v[i] = x.v[i] + acc.v[i];
      stv<T, V, NT>(px, x);
    }
  }
}

// ---- 27-point consumer on Cartesian blocks with a one-cell halo ----------------------------
struct StDesc {
  int32_t nblk, nz, ny, nx;
  int64_t sz, sy;       // cell strides of a block's full box
  int64_t bcells;       // cells per block full box
  const int64_t* info;  // per block, 27 directions: source block, -1 zero, -2 own ghost
};

// 27-point operator, LDS-tiled.  A workgroup owns a 64 (x) x 8 (y) column of
// outputs over ST_ZC planes and marches in z: each (x, y) plane of the tile
// with its one-cell halo (66 x 10 values) is staged in LDS, the 3x3 plane sums
// are formed separably (3 along x, then 3 along y), and
// y = 27 x_c - (S(z-1) + S(z) + S(z+1)) = 26 x_c - (sum of the 26 neighbours).
// Two planes of global loads are in flight while one is summed (register sets
// A and B), and every memory instruction of the march is issued
// unconditionally: loads take clamped addresses and drop the value, stores go
// through buffer resources with an out-of-range offset where a lane stores
// nothing.  Loads and stores retire from one in-order counter, so a guarded
// instruction would make the compiler wait for everything issued before the
// plane it needs (earlier stores included); straight-line code lets each wait
// cover only that plane.
// FUSED: values outside a block's data box come through the BC (the source
// block's data cell for halo copies, zero for zero rows, x itself where the
// BC writes nothing).  GHOSTS: each ghost value read through the BC is also
// stored into x by the one tile that owns it (the tile whose data range holds
// the ghost's position clamped into the data box), which leaves x's covered
// ghosts as the BC's apply would.
constexpr int ST_TX = 64, ST_TY = 8, ST_ZC = 32;
constexpr int ST_RPT = ST_TY / 4;  // output rows per thread (4 wavefronts of 64 columns)
constexpr int ST_LX = ST_TX + 2, ST_LY = ST_TY + 2, ST_PLANE = ST_LX * ST_LY;
constexpr int ST_NLOAD = (ST_LY * ST_TX + 255) / 256;  // interior columns of the TY + 2 rows
constexpr int ST_NS = ST_NLOAD + 1;                     // + one value of the two halo columns
constexpr int ST_LDS = ST_PLANE + 256;                  // + one slot per thread for values with no place
static_assert(ST_TY % 4 == 0, "tile rows must split over 4 wavefronts");

// One value a thread fetches per plane: column (y, xx) of the block's halo box.
struct StSlot {
  int y, xx;   // block-local position (clamped into the halo box where !valid)
  int dy, dx;  // -1, 0, 1: below, inside, above the data range
  int lds;     // LDS slot
  bool valid;  // a position of the tile's halo box inside the block's halo box
  bool own;    // this tile stores ghosts of this column (its clamped position lies in the tile)
};

__device__ __forceinline__ int st_dir(int v, int n) { return v < 0 ? -1 : (v >= n ? 1 : 0); }

// k < ST_NLOAD: interior columns of the TY + 2 rows (element e = thread + 256 k,
// one row per wavefront access); k == ST_NLOAD: the two halo columns
// (threads 0 .. 2 (TY + 2) - 1).
__device__ __forceinline__ StSlot st_slot(const StDesc& st, int k, int y0, int x0) {
  StSlot s;
  const int t = threadIdx.x;
  int ly, lx;
  if (k < ST_NLOAD) {
    const int e = t + k * 256;
    ly = e >> 6;
    lx = (e & 63) + 1;
    s.valid = e < ST_LY * ST_TX;
    s.lds = s.valid ? ly * ST_LX + lx : ST_PLANE + t;
  } else {
    const bool h = t < 2 * ST_LY;
    ly = h ? t >> 1 : 0;
    lx = h && (t & 1) ? ST_LX - 1 : 0;
    s.valid = h;
    s.lds = h ? ly * ST_LX + lx : ST_PLANE + t;
  }
  const int y = y0 + ly - 1, xx = x0 + lx - 1;  // xx == nx / y == ny: the far halo of a partial tile
  s.valid = s.valid && y <= st.ny && xx <= st.nx;
  s.y = min(y, st.ny);
  s.xx = min(xx, st.nx);
  s.dy = st_dir(s.y, st.ny);
  s.dx = st_dir(s.xx, st.nx);
  const int cy = min(max(s.y, 0), st.ny - 1), cx = min(max(s.xx, 0), st.nx - 1);
  s.own = s.valid && cy >= y0 && cy < y0 + ST_TY && cx >= x0 && cx < x0 + ST_TX;
  return s;
}

template <typename T, int AUX>
__device__ __forceinline__ void st_buf_store(T v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
  if constexpr (sizeof(T) == 8) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, AUX);
  } else {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, AUX);
  }
}

// Issue the loads of plane z into one register set.  keep: bit k set where
// value k is used as loaded (a valid position that is not a zero row).
// goff: byte offsets of the ghost stores in the chunk's x resource (BUF_OOB: none).
template <typename T, bool FUSED, bool GHOSTS>
__device__ __forceinline__ void st_fetch(const T* __restrict__ x, const StDesc& st, const int64_t* info, int b,
                                         int z, int z0, int z1, const StSlot (&sl)[ST_NS], T (&v)[ST_NS],
                                         uint32_t& keep, uint32_t (&goff)[ST_NS]) {
  const int dz = st_dir(z, st.nz);
  // ghosts of plane z belong to this chunk when z is a z ghost (only the first
  // or last chunk reads it) or one of the chunk's own planes
  const bool zown = dz != 0 || (z >= z0 && z < z1);
  keep = 0;
#pragma unroll
  for (int k = 0; k < ST_NS; ++k) {
    int64_t blk = b;
    int zz = z, yy = sl[k].y, xx = sl[k].xx;
    bool zero = false, covered = false;
    const bool ghost = dz != 0 || sl[k].dy != 0 || sl[k].dx != 0;
    if (FUSED && ghost) {
      const int64_t o = info[(dz + 1) * 9 + (sl[k].dy + 1) * 3 + (sl[k].dx + 1)];
      covered = o != -2;
      zero = o == -1;
      if (o >= 0) {
        blk = o;
        zz -= dz * st.nz;
        yy -= sl[k].dy * st.ny;
        xx -= sl[k].dx * st.nx;
      }
    }
    v[k] = x[blk * st.bcells + (int64_t)(zz + 1) * st.sz + (int64_t)(yy + 1) * st.sy + (xx + 1)];
    if (sl[k].valid && !zero) keep |= 1u << k;
    if (GHOSTS) {
      const bool g = sl[k].own && ghost && covered && zown;
      goff[k] = g ? (uint32_t)(((int64_t)(z + 1 - z0) * st.sz + (int64_t)(sl[k].y + 1) * st.sy + (sl[k].xx + 1)) *
                               (int64_t)sizeof(T))
                  : BUF_OOB;
    }
  }
}

// One LDS write per value (values with no place go to the thread's spare
// slot) and, with GHOSTS, one buffer store per value (dropped where goff is
// out of range).
template <typename T, bool GHOSTS>
__device__ __forceinline__ void st_put(T* plane, const StSlot (&sl)[ST_NS], const T (&v)[ST_NS], uint32_t keep,
                                       const uint32_t (&goff)[ST_NS], __amdgpu_buffer_rsrc_t xr) {
#pragma unroll
  for (int k = 0; k < ST_NS; ++k) {
    const T val = (keep >> k) & 1u ? v[k] : T(0);
    plane[sl[k].lds] = val;
    if (GHOSTS) st_buf_store<T, 0>(val, xr, goff[k]);
  }
}

// One launch of stencil tiles.  Workgroups are dealt to the 8 XCDs
// round-robin; tiles are renumbered so that each XCD gets a contiguous run of
// them (neighbouring tiles share halo rows in its L2).  Per-chunk buffer
// ranges stay below 2 GiB (checked by the host).
template <typename T, bool FUSED, bool GHOSTS>
__global__ __launch_bounds__(256) void k_stencil27(const T* __restrict__ x, T* xg, T* __restrict__ yout,
                                                   StDesc st) {
  static_assert(FUSED || !GHOSTS, "ghost stores need the fused form");
  __shared__ T buf[2][ST_LDS];
  __shared__ int64_t info[27];  // this block's direction table, read once
  const int ntx = (st.nx + ST_TX - 1) / ST_TX, nty = (st.ny + ST_TY - 1) / ST_TY, nzc = (st.nz + ST_ZC - 1) / ST_ZC;
  const int nst = ntx * nty * nzc * st.nblk;
  int bid;
  {
    const int q = nst >> 3, rem = nst & 7, xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    bid = xcd * q + min(xcd, rem) + j;
  }
  const int tile_x = bid % ntx;
  bid /= ntx;
  const int tile_y = bid % nty;
  bid /= nty;
  const int tile_z = bid % nzc;
  const int b = bid / nzc;
  if (b >= st.nblk) return;  // uniform per workgroup
  const int x0 = tile_x * ST_TX, y0 = tile_y * ST_TY, z0 = tile_z * ST_ZC, z1 = min(z0 + ST_ZC, st.nz);
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // each thread: column tx, rows RPT*ty ..
  if (FUSED) {
    if (threadIdx.x < 27) info[threadIdx.x] = st.info[b * 27 + threadIdx.x];
    __syncthreads();
  }
  StSlot sl[ST_NS];
#pragma unroll
  for (int k = 0; k < ST_NS; ++k) sl[k] = st_slot(st, k, y0, x0);
  const int64_t plane_out = (int64_t)st.ny * st.nx;
  // y: this chunk's planes of block b; x (ghost stores): its planes z0 - 1 .. z1
  const __amdgpu_buffer_rsrc_t yr = __builtin_amdgcn_make_buffer_rsrc(
      yout + ((int64_t)b * st.nz + z0) * plane_out, 0, (int)((z1 - z0) * plane_out * (int64_t)sizeof(T)),
      BUF_RSRC_WORD3);
  __amdgpu_buffer_rsrc_t xr = yr;
  if (GHOSTS)
    xr = __builtin_amdgcn_make_buffer_rsrc(xg + b * st.bcells + (int64_t)z0 * st.sz, 0,
                                           (int)((z1 - z0 + 2) * st.sz * (int64_t)sizeof(T)), BUF_RSRC_WORD3);
  T A[ST_NS], B[ST_NS];
  uint32_t ka, kb, ga[ST_NS], gb[ST_NS];
  // plane z0 - 1 goes straight to LDS buffer 0; planes z0 and z0 + 1 go in flight
  st_fetch<T, FUSED, GHOSTS>(x, st, info, b, z0 - 1, z0, z1, sl, A, ka, ga);
  st_put<T, GHOSTS>(buf[0], sl, A, ka, ga, xr);
  st_fetch<T, FUSED, GHOSTS>(x, st, info, b, z0, z0, z1, sl, A, ka, ga);
  st_fetch<T, FUSED, GHOSTS>(x, st, info, b, min(z0 + 1, z1), z0, z1, sl, B, kb, gb);
  __syncthreads();
  T sm2[ST_RPT], sm1[ST_RPT], cm1[ST_RPT];
#pragma unroll
  for (int q = 0; q < ST_RPT; ++q) sm2[q] = sm1[q] = cm1[q] = T(0);
  // One step: LDS holds plane p; sum it, store y(p - 1) (STORE), put plane
  // p + 1 from the set S into the other LDS buffer (PUT), then reuse S for
  // plane p + 3 (clamped to z1: a spare load keeps the instruction count fixed).
  auto step = [&](int p, T(&S)[ST_NS], uint32_t& kS, uint32_t(&gS)[ST_NS], auto store_c, auto put_c) {
    constexpr bool STORE = decltype(store_c)::value, PUT = decltype(put_c)::value;
    const int cur = (p - z0 + 1) & 1;
    T hsum[ST_RPT + 2];
#pragma unroll
    for (int q = 0; q < ST_RPT + 2; ++q) {
      const T* row = &buf[cur][(ST_RPT * ty + q) * ST_LX + tx];
      hsum[q] = (row[0] + row[1]) + row[2];
    }
    T sn[ST_RPT], cn[ST_RPT], yv[ST_RPT];
#pragma unroll
    for (int q = 0; q < ST_RPT; ++q) {
      sn[q] = (hsum[q] + hsum[q + 1]) + hsum[q + 2];
      cn[q] = buf[cur][(ST_RPT * ty + q + 1) * ST_LX + tx + 1];
      yv[q] = T(27) * cm1[q] - ((sm2[q] + sm1[q]) + sn[q]);
      sm2[q] = sm1[q];
      sm1[q] = sn[q];
      cm1[q] = cn[q];
    }
    if constexpr (PUT) st_put<T, GHOSTS>(buf[cur ^ 1], sl, S, kS, gS, xr);
    if constexpr (STORE) {
#pragma unroll
      for (int q = 0; q < ST_RPT; ++q) {
        const int yy = y0 + ST_RPT * ty + q, xx = x0 + tx;
        const uint32_t off = yy < st.ny && xx < st.nx
                                 ? (uint32_t)(((int64_t)(p - 1 - z0) * plane_out + (int64_t)yy * st.nx + xx) *
                                              (int64_t)sizeof(T))
                                 : BUF_OOB;
        st_buf_store<T, 2>(yv[q], yr, off);  // non-temporal
      }
    }
    if constexpr (PUT) {
      __syncthreads();
      st_fetch<T, FUSED, GHOSTS>(x, st, info, b, min(p + 3, z1), z0, z1, sl, S, kS, gS);
    }
  };
  using Y = std::true_type;
  using N = std::false_type;
  step(z0 - 1, A, ka, ga, N{}, Y{});  // plane z0 from A
  step(z0, B, kb, gb, N{}, Y{});      // plane z0 + 1 from B
  int p = z0 + 1;
  for (; p + 1 <= z1 - 1; p += 2) {
    step(p, A, ka, ga, Y{}, Y{});
    step(p + 1, B, kb, gb, Y{}, Y{});
  }
  if (p <= z1 - 1) {
    step(p, A, ka, ga, Y{}, Y{});
    ++p;
  }
  step(p, A, ka, ga, Y{}, N{});  // p == z1: the last output plane z1 - 1
}

// ---- consumer of the BC's ghosts (stencil of offsets and weights) --------------------
// Structured tiles: a run of cells along the last dimension, which each row
// group walks in one of three ways (the line walk, the pipelined walk, or
// batches of CONS_RB cells with the offsets EC at a time; see k_consumer),
// every sum in the consumer's offset order (first product, then FMAs).
// Boundary rows (fused form): the stencil composed with the BC rows of the
// ghosts it reaches, as entries (cell, weight, component rotation) summed in
// order, plus the composed b.  The output y holds the data cells block by block, each block's
// data box row-major, inner values point-major.
struct ConsDesc {
  const int32_t* delta;  // per block: noff cell deltas
  const void* w;         // noff weights
  int32_t noff;
  int32_t ntiles;
  const CTile* tiles;
  const int32_t* brow_y;
  const int32_t* bptr;
  const int32_t* bcol;
  const void* bw;
  const int8_t* brot;
  const int32_t* bconst_row;
  const void* bconst;
  int32_t nbrow;  // boundary rows (0: unfused)
  int32_t tile_rows;  // boundary rows per tile
  void* y;
  const int32_t* line_delta;  // line walk: per block, cell delta of each line's last point
  const void* line_w;         // lines x 3 ring-slot weights
  int32_t line_mask;          // bit 3 l + s: slot s of line l is an offset
};

// Line walk of a structured tile (NL lines, see ConsumerHost): slot s of
// line l's ring holds the point k + line_delta[l] - 2 + s of cell k.  A row
// group walks its cells in chunks of CONS_CELLS steps; every step issues the
// next cell's new point of each line before the current cell's sum and
// store, and every load and store is issued whatever the chunk's length
// (loads clamped to the chunk's last cell, stores past it dropped through
// the output range), so that each wait is for the current cell's points only.
template <typename T, int V, bool NT, int NL>
__device__ __forceinline__ void cons_lines(const PlanDesc& d, const ConsDesc& c, const CTile& t, int kb, int ke,
                                           int lane) {
  constexpr int NS = CONS_CELLS;
  const T* __restrict__ x = static_cast<const T*>(d.field);
  const int64_t l = (int64_t)lane * V;
  const int32_t* __restrict__ ld = c.line_delta + (int64_t)t.blk * NL;
  const T* __restrict__ lw = static_cast<const T*>(c.line_w);
  int32_t dl[NL], s0[NL];
  T w[NL][3];
  bool on[NL][3];
#pragma unroll
  for (int q = 0; q < NL; ++q) {
    dl[q] = ld[q];
    const int m3 = (c.line_mask >> (3 * q)) & 7;
    s0[q] = (m3 & 1) ? 0 : ((m3 & 2) ? 1 : 2);  // the line's first slot (slots before it are never read)
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      w[q][u] = lw[3 * q + u];
      on[q][u] = (m3 >> u) & 1;
    }
  }
  const T* __restrict__ xb = x + (int64_t)t.cell0 * d.cs + l;
  const int row_bytes = (int)(d.inner * (int64_t)sizeof(T));
  for (int k0 = kb; k0 < ke; k0 += NS) {
    const int last = min(ke, k0 + NS) - 1;
    Pack<T, V> R[NL][3];
#pragma unroll
    for (int q = 0; q < NL; ++q)
#pragma unroll
      for (int u = 0; u < 3; ++u) R[q][u] = ldv<T, V>(xb + (int64_t)(k0 + dl[q] - 2 + max(u, s0[q])) * d.cs);
    // the chunk's output rows: one buffer range (NS rows of at most 4 KiB each: a
    // one-pass row group covers at most 256 lanes of 16 bytes)
    T* yc = static_cast<T*>(c.y) + (int64_t)(t.y0 + k0) * d.inner;
    const __amdgpu_buffer_rsrc_t yr =
        __builtin_amdgcn_make_buffer_rsrc(yc, 0, (last - k0 + 1) * row_bytes, BUF_RSRC_WORD3);
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      const int kn = min(k0 + j + 1, last);
      Pack<T, V> nx[NL];
#pragma unroll
      for (int q = 0; q < NL; ++q) nx[q] = ldv<T, V>(xb + (int64_t)(kn + dl[q]) * d.cs);
      Pack<T, V> acc;
#pragma unroll
      for (int i = 0; i < V; ++i) acc.v[i] = T(-0.0);  // fma(w, x, -0) = w * x: the first term is a product
#pragma unroll
      for (int q = 0; q < NL; ++q)
#pragma unroll
        for (int u = 0; u < 3; ++u)
#pragma unroll
          for (int i = 0; i < V; ++i) acc.v[i] = on[q][u] ? fma(w[q][u], R[q][u].v[i], acc.v[i]) : acc.v[i];
      const uint32_t off = (uint32_t)((int64_t)j * d.inner + l) * (uint32_t)sizeof(T);
      stv_buf<T, V, NT>(acc, yr, k0 + j <= last ? off : BUF_OOB);
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        R[q][0] = R[q][1];
        R[q][1] = R[q][2];
        R[q][2] = nx[q];
      }
    }
  }
}

// WALK of the structured tiles: 0, the offsets 8 at a time over a batch of
// cells; 1, the pipelined walk (at most 8 offsets, one pass of a row group
// per cell); 10 + NL, the line walk of NL lines (one pass per cell).  The
// boundary rows' tiles come first in the grid (they then overlap the
// structured tiles instead of trailing them).
template <typename T, int V, bool NT, int WALK>
__global__ __launch_bounds__(256) void k_consumer(PlanDesc d, ConsDesc c) {
  constexpr int RB = CONS_RB, EC = 8;
  const int lpr = 1 << d.lpr_shift;
  const int ngroups = (int)blockDim.x >> d.lpr_shift;
  const int grp = (int)threadIdx.x >> d.lpr_shift, lane = (int)threadIdx.x & (lpr - 1);
  const T* __restrict__ x = static_cast<const T*>(d.field);
  T* __restrict__ y = static_cast<T*>(c.y);
  const int64_t nvec = d.inner / V;
  const int nbt = (c.nbrow + c.tile_rows - 1) / c.tile_rows;
  if ((int)blockIdx.x >= nbt) {
    // workgroups are dealt to the 8 XCDs round-robin: give each XCD a
    // contiguous band of tiles, so the rows a cell's neighbours share were
    // read shortly before into that XCD's L2
    int b = (int)blockIdx.x - nbt;
    {
      const int q = c.ntiles >> 3, rem = c.ntiles & 7, xcd = b & 7, jx = b >> 3;
      b = xcd * q + min(xcd, rem) + jx;
    }
    const CTile t = c.tiles[b];
    const int32_t* __restrict__ dl = c.delta + (int64_t)t.blk * c.noff;
    const T* __restrict__ w = static_cast<const T*>(c.w);
    // a row group walks a contiguous part of the tile's run
    const int cpg = (t.n + ngroups - 1) / ngroups;
    const int kb = grp * cpg, ke = min(t.n, kb + cpg);
    if constexpr (WALK > 10) {
      if (lane < nvec && kb < ke) cons_lines<T, V, NT, WALK - 10>(d, c, t, kb, ke, lane);
      return;
    } else if constexpr (WALK == 1) {
      // one pass per cell: the next cell's reads issued before the current
      // cell's store (two register sets, A and B)
      if (lane >= nvec) return;
      const int64_t l = (int64_t)lane * V;
      int32_t dm[EC];
      T wm[EC];
#pragma unroll
      for (int m = 0; m < EC; ++m) {
        dm[m] = m < c.noff ? dl[m] : 0;
        wm[m] = m < c.noff ? w[m] : T(0);
      }
      const T* xb = x + (int64_t)t.cell0 * d.cs + l;
      Pack<T, V> A[EC], B[EC];
      auto issue = [&](Pack<T, V> (&buf)[EC], int k) {
#pragma unroll
        for (int m = 0; m < EC; ++m)
          if (m < c.noff) buf[m] = ldv<T, V>(xb + (int64_t)(k + dm[m]) * d.cs);
      };
      auto finish = [&](Pack<T, V> (&buf)[EC], int k) {
        Pack<T, V> acc;
#pragma unroll
        for (int m = 0; m < EC; ++m)
          if (m < c.noff) {
#pragma unroll
            for (int i = 0; i < V; ++i) acc.v[i] = m == 0 ? wm[m] * buf[m].v[i] : fma(wm[m], buf[m].v[i], acc.v[i]);
          }
        stv<T, V, NT>(y + (int64_t)(t.y0 + k) * d.inner + l, acc);
      };
      if (kb < ke) issue(A, kb);
      for (int k = kb; k < ke; k += 2) {
        if (k + 1 < ke) issue(B, k + 1);
        finish(A, k);
        if (k + 1 < ke) {
          if (k + 2 < ke) issue(A, k + 2);
          finish(B, k + 1);
        }
      }
      return;
    } else {
    for (int k0 = kb; k0 < ke; k0 += RB)
      for (int64_t v = lane; v < nvec; v += lpr) {
        const int64_t l = v * V;
        Pack<T, V> acc[RB];
        for (int e0 = 0; e0 < c.noff; e0 += EC) {
          Pack<T, V> xv[RB][EC];
#pragma unroll
          for (int q = 0; q < RB; ++q)
            if (k0 + q < ke)
#pragma unroll
              for (int m = 0; m < EC; ++m)
                if (e0 + m < c.noff) xv[q][m] = ldv<T, V>(x + (int64_t)(t.cell0 + k0 + q + dl[e0 + m]) * d.cs + l);
#pragma unroll
          for (int q = 0; q < RB; ++q)
#pragma unroll
            for (int m = 0; m < EC; ++m)
              if (e0 + m < c.noff) {
                const T wv = w[e0 + m];
#pragma unroll
                for (int i = 0; i < V; ++i)
                  acc[q].v[i] = e0 + m == 0 ? wv * xv[q][m].v[i] : fma(wv, xv[q][m].v[i], acc[q].v[i]);
              }
        }
#pragma unroll
        for (int q = 0; q < RB; ++q)
          if (k0 + q < ke) stv<T, V, NT>(y + (int64_t)(t.y0 + k0 + q) * d.inner + l, acc[q]);
      }
    }
    return;
  }
  // boundary rows: a row group takes one row at a time, EC entries' loads
  // in flight, summed in entry order
  const T* __restrict__ bw = static_cast<const T*>(c.bw);
  const T* __restrict__ bc = static_cast<const T*>(c.bconst);
  const int r0 = (int)blockIdx.x * c.tile_rows;
  const int r1 = min(c.nbrow, r0 + c.tile_rows);
  for (int r = r0 + grp; r < r1; r += ngroups)
    for (int64_t v = lane; v < nvec; v += lpr) {
      const int64_t l = v * V;
      const int eb = c.bptr[r], ee = c.bptr[r + 1];
      Pack<T, V> acc;
#pragma unroll
      for (int i = 0; i < V; ++i) acc.v[i] = T(0);
      for (int j0 = eb; j0 < ee; j0 += EC) {
        Pack<T, V> xv[EC];
        T wv[EC];
#pragma unroll
        for (int m = 0; m < EC; ++m) {
          wv[m] = T(0);
          if (j0 + m < ee) {
            T sign;
            const int64_t sl = rot_slot<T>(d, c.brot[j0 + m], l, sign);
            wv[m] = bw[j0 + m] * sign;
            xv[m] = ldv<T, V>(x + (int64_t)c.bcol[j0 + m] * d.cs + sl);
          }
        }
#pragma unroll
        for (int m = 0; m < EC; ++m)
          if (j0 + m < ee) {
#pragma unroll
            for (int i = 0; i < V; ++i)
              acc.v[i] = j0 + m == eb ? wv[m] * xv[m].v[i] : fma(wv[m], xv[m].v[i], acc.v[i]);
          }
      }
      const int br = c.bconst_row[r];
      if (br >= 0)
#pragma unroll
        for (int i = 0; i < V; ++i) acc.v[i] = acc.v[i] + bc[(int64_t)br * d.inner + l + i];
      stv<T, V, NT>(y + (int64_t)c.brow_y[r] * d.inner + l, acc);
    }
}


// ---- FP64 cubed-sphere interpolation weights ------------------------------------------
// Ghost layer k beyond an edge, tangential index t: the ray through the ghost
// meets the neighbour face on its grid line at distance k from the edge, at
// tangential angle atan(tan(beta_t) / tan(pi/4 + (k + 1/2) D)), D = pi / 2N.
__global__ void k_cs_weights(int N, int h, int32_t* __restrict__ base, double* __restrict__ w) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= h * N) return;
  const int k = idx / N, t = idx % N;
  const double q = M_PI / 4.0;
  const double D = M_PI / (2.0 * N);
  const double ta = tan(q + (k + 0.5) * D);
  const double tb = tan(-q + (t + 0.5) * D);
  double s = (atan(tb / ta) + q) / D - 0.5;
  const double rs = rint(s);
  if (fabs(s - rs) <= 1e-9) s = rs;
  int b0 = (int)floor(s) - 1;
  b0 = b0 < 0 ? 0 : (b0 > N - 4 ? N - 4 : b0);
  const double d0 = s - b0, d1 = s - (b0 + 1), d2 = s - (b0 + 2), d3 = s - (b0 + 3);
  base[idx] = b0;
  w[4 * idx + 0] = -d1 * d2 * d3 / 6.0;
  w[4 * idx + 1] = d0 * d2 * d3 / 2.0;
  w[4 * idx + 2] = -d0 * d1 * d3 / 2.0;
  w[4 * idx + 3] = d0 * d1 * d2 / 6.0;
}

// ---- device tables -------------------------------------------------------------------------
namespace {

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

// Slice width of the wide-row kernel: 256 bytes (lanes of four FP64 values)
// for FP64 plans of at least 32 inner values whose layout is 4-aligned, else
// 128 bytes.
static int wide_slice_bytes(const Plan& p) {
  const Layout& L = p.layout;
  const bool a4 = L.inner % 4 == 0 && (L.vec_len == 0 || (L.vec_lo % 4 == 0 && L.vec_stride % 4 == 0 &&
                                                          L.vec_len % 4 == 0));
  return p.dtype == HBC_F64 && L.order == HBC_POINT_MAJOR && a4 && L.inner >= 32 ? 2 * WIDE_ROW_BYTES
                                                                                  : WIDE_ROW_BYTES;
}

struct Packer {
  std::vector<char> buf;
  size_t put(const void* p, size_t n) {
    size_t off = align256(buf.size());
    buf.resize(off + align256(std::max<size_t>(n, 1)));
    if (n) std::memcpy(buf.data() + off, p, n);
    return off;
  }
  template <class V>
  size_t vec(const V& v) {
    return put(v.data(), v.size() * sizeof(typename V::value_type));
  }
  size_t reals(const std::vector<double>& v, int dtype) {
    if (dtype == HBC_F64) return vec(v);
    std::vector<float> f(v.size());
    for (size_t k = 0; k < v.size(); ++k) f[k] = (float)v[k];  // round to nearest
    return vec(f);
  }
  // wide-row entries as WideEnt<T>: the weight in the plan's type (rounded as
  // in reals) and the LDS offset of the source cell's slice (slot * values
  // per slice of sb bytes)
  size_t wide_entries(const std::vector<double>& w, const std::vector<int32_t>& slot, int dtype, int sb) {
    if (dtype == HBC_F64) {
      std::vector<WideEnt<double>> e(w.size());
      for (size_t k = 0; k < w.size(); ++k) e[k] = {w[k], slot[k] * (sb / 8)};
      return vec(e);
    }
    std::vector<WideEnt<float>> e(w.size());
    for (size_t k = 0; k < w.size(); ++k) e[k] = {(float)w[k], slot[k] * (sb / 4)};
    return vec(e);
  }
};

int ilog2(int v) {
  int s = 0;
  while ((1 << s) < v) ++s;
  return s;
}

PlanDesc make_desc(const Plan& p, void* field) {
  PlanDesc d{};
  d.field = field;
  d.segs = p.d_segs;
  d.ell_col = p.d_ell_col;
  d.ell_val = p.d_ell_val;
  d.csr_ptr = p.d_csr_ptr;
  d.csr_col = p.d_csr_col;
  d.csr_val = p.d_csr_val;
  d.bval = p.d_bval;
  d.row_dst = p.d_row_dst;
  d.row_src = p.d_row_src;
  d.inner = p.layout.inner;
  if (p.layout.order == HBC_POINT_MAJOR) {
    d.cs = p.layout.inner;
    d.ls = 1;
  } else {
    d.cs = 1;
    d.ls = p.grid.ncells;
  }
  d.vec_lo = p.layout.vec_lo;
  d.vec_stride = p.layout.vec_stride;
  d.vec_len = p.layout.vec_len;
  d.lpr_shift = ilog2(p.tune.lanes_per_row);
  d.vec = p.vec;
  d.chunked = p.tune.lanes_per_row >= CHUNK_LPR ? 1 : 0;
  d.nt = (p.layout.order == HBC_POINT_MAJOR && p.layout.inner * (p.dtype == HBC_F64 ? 8 : 4) >= 128) ? 1 : 0;
  d.unroll = p.unroll;
  d.general = 0;
  for (const RowTile& t : p.host.rtiles)
    if (t.kind == SEG_CSR || (t.kind == SEG_ELL && (t.width != 4 || (t.flags & SEGF_ELL_PADDED)))) d.general = 1;
  // rows of a length that 16-byte vectors do not divide, with no vector
  // components to rotate and no data rows (whose gather assumes whole vectors)
  const int64_t vfull = p.dtype == HBC_F64 ? 2 : 4;
  d.ua = p.layout.order == HBC_POINT_MAJOR && p.layout.vec_len == 0 && p.stats.rows_data == 0 &&
         p.layout.inner % vfull != 0 && p.layout.inner > vfull;
  return d;
}

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

}  // namespace

void device_free_plan(Plan& p) {
  if (p.dev) (void)hipFree(p.dev);
  p.dev = nullptr;
  p.dev_bytes = 0;
  if (p.d_st_dev) (void)hipFree(p.d_st_dev);
  p.d_st_dev = nullptr;
  p.d_st_info = nullptr;
  if (p.d_adj_tiles) (void)hipFree(const_cast<AdjTile*>(p.d_adj_tiles));
  p.d_adj_tiles = nullptr;
  if (p.d_csc_dev) (void)hipFree(p.d_csc_dev);
  p.d_csc_dev = nullptr;
  if (p.d_al_dev) (void)hipFree(p.d_al_dev);
  p.d_al_dev = nullptr;
  if (p.d_dr_scratch) (void)hipFree(p.d_dr_scratch);
  p.d_dr_scratch = nullptr;
  p.d_csc_src = nullptr;
  if (p.d_tiles) (void)hipFree(const_cast<DevTile*>(p.d_tiles));
  p.d_tiles = nullptr;
}

void device_upload_plan(Plan& p) {
  Packer pk;
  const HostTables& T = p.host;
  size_t o_segs = pk.vec(T.segs);
  size_t o_ellc = pk.vec(T.ell_col);
  size_t o_ellv = pk.reals(T.ell_val, p.dtype);
  size_t o_csrp = pk.vec(T.csr_ptr);
  size_t o_csrc = pk.vec(T.csr_col);
  size_t o_csrv = pk.reals(T.csr_val, p.dtype);
  size_t o_b = pk.reals(T.bval, p.dtype);
  size_t o_rd = pk.vec(T.row_dst);
  size_t o_rs = pk.vec(T.row_src);
  size_t o_wt = pk.vec(T.wtiles);
  size_t o_wu = pk.vec(T.w_ucell);
  size_t o_wr = pk.vec(T.w_row);
  size_t o_wp = pk.vec(T.w_rp);
  size_t o_we = pk.wide_entries(T.w_entw, T.w_ents, p.dtype, wide_slice_bytes(p));
  size_t o_nt = pk.vec(T.ntiles);
  size_t o_drc = pk.vec(T.dr_cell);
  size_t o_drp = pk.vec(T.dr_ptr);
  size_t o_drk = pk.vec(T.dr_col);
  size_t o_drv = pk.reals(T.dr_val, p.dtype);
  size_t o_dcc = pk.vec(T.dc_comp);
  size_t o_dcd = pk.vec(T.dc_row_dst);
  size_t o_dce = pk.vec(T.dc_row_ent);
  size_t o_dcn = pk.vec(T.dc_row_n);
  size_t o_dcs = pk.vec(T.dc_slot);
  size_t o_dcw = pk.reals(T.dc_w, p.dtype);
  void* dev = nullptr;
  hipError_t e = hipMalloc(&dev, pk.buf.size());
  if (e != hipSuccess) fail(e == hipErrorOutOfMemory ? HBC_ENOMEM : HBC_EHIP, std::string("hipMalloc: ") + hipGetErrorString(e));
  p.dev = dev;
  p.dev_bytes = pk.buf.size();
  HIP_CHECK(hipMemcpy(dev, pk.buf.data(), pk.buf.size(), hipMemcpyHostToDevice));
  char* b = static_cast<char*>(dev);
  p.d_segs = reinterpret_cast<const DevSeg*>(b + o_segs);
  p.d_ell_col = reinterpret_cast<const int32_t*>(b + o_ellc);
  p.d_ell_val = b + o_ellv;
  p.d_csr_ptr = reinterpret_cast<const int64_t*>(b + o_csrp);
  p.d_csr_col = reinterpret_cast<const int32_t*>(b + o_csrc);
  p.d_csr_val = b + o_csrv;
  p.d_bval = b + o_b;
  p.d_row_dst = reinterpret_cast<const int32_t*>(b + o_rd);
  p.d_row_src = reinterpret_cast<const int32_t*>(b + o_rs);
  p.d_wtiles = reinterpret_cast<const WideTile*>(b + o_wt);
  p.d_w_ucell = reinterpret_cast<const int32_t*>(b + o_wu);
  p.d_w_row = reinterpret_cast<const int32_t*>(b + o_wr);
  p.d_w_rp = reinterpret_cast<const int32_t*>(b + o_wp);
  p.d_w_ent = b + o_we;
  p.d_ntiles = reinterpret_cast<const NarrowTile*>(b + o_nt);
  p.d_dr_cell = reinterpret_cast<const int32_t*>(b + o_drc);
  p.d_dr_ptr = reinterpret_cast<const int64_t*>(b + o_drp);
  p.d_dr_col = reinterpret_cast<const int32_t*>(b + o_drk);
  p.d_dr_val = b + o_drv;
  p.d_dc_comp = reinterpret_cast<const DataComp*>(b + o_dcc);
  p.d_dc_row_dst = reinterpret_cast<const int32_t*>(b + o_dcd);
  p.d_dc_row_ent = reinterpret_cast<const int32_t*>(b + o_dce);
  p.d_dc_row_n = reinterpret_cast<const int32_t*>(b + o_dcn);
  p.d_dc_slot = reinterpret_cast<const int32_t*>(b + o_dcs);
  p.d_dc_w = b + o_dcw;
  if (p.stats.rows_data > 0 && !T.dc_ok) {
    void* sc = nullptr;
    const size_t n = (size_t)p.stats.rows_data * (size_t)p.layout.inner * (p.dtype == HBC_F64 ? 8 : 4);
    e = hipMalloc(&sc, n);
    if (e != hipSuccess) fail(e == hipErrorOutOfMemory ? HBC_ENOMEM : HBC_EHIP, std::string("hipMalloc: ") + hipGetErrorString(e));
    p.d_dr_scratch = sc;
  }
  device_upload_tiles(p);
  if (p.st_fused) {
    void* si = nullptr;
    HIP_CHECK(hipMalloc(&si, p.st_info.size() * sizeof(int64_t)));
    p.d_st_dev = si;
    HIP_CHECK(hipMemcpy(si, p.st_info.data(), p.st_info.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    p.d_st_info = static_cast<const int64_t*>(si);
  }
}

void device_upload_tiles(Plan& p) {
  // one allocation: segment tiles (plane-major path), then row tiles (point-major path)
  if (p.d_tiles) HIP_CHECK(hipFree(const_cast<DevTile*>(p.d_tiles)));
  p.d_tiles = nullptr;
  p.d_rtiles = nullptr;
  p.d_wruns = nullptr;
  ++p.tile_gen;  // graphs captured before this point hold the old tables
  const size_t n1 = align256(std::max<size_t>(1, p.host.tiles.size()) * sizeof(DevTile));
  const size_t n2 = align256(std::max<size_t>(1, p.host.rtiles.size()) * sizeof(RowTile));
  const size_t n3 = std::max<size_t>(1, p.host.wruns.size()) * sizeof(WinRun);
  void* t = nullptr;
  HIP_CHECK(hipMalloc(&t, n1 + n2 + n3));
  if (!p.host.tiles.empty())
    HIP_CHECK(hipMemcpy(t, p.host.tiles.data(), p.host.tiles.size() * sizeof(DevTile), hipMemcpyHostToDevice));
  if (!p.host.rtiles.empty())
    HIP_CHECK(hipMemcpy(static_cast<char*>(t) + n1, p.host.rtiles.data(), p.host.rtiles.size() * sizeof(RowTile),
                        hipMemcpyHostToDevice));
  if (!p.host.wruns.empty())
    HIP_CHECK(hipMemcpy(static_cast<char*>(t) + n1 + n2, p.host.wruns.data(), p.host.wruns.size() * sizeof(WinRun),
                        hipMemcpyHostToDevice));
  p.d_tiles = static_cast<const DevTile*>(t);
  p.d_rtiles = reinterpret_cast<const RowTile*>(static_cast<char*>(t) + n1);
  p.d_wruns = reinterpret_cast<const WinRun*>(static_cast<char*>(t) + n1 + n2);
}

void device_upload_csc(Plan& p) {
  Packer pk;
  const CscHost& C = p.host.csc;
  size_t o_src = pk.vec(C.src_cell);
  size_t o_ptr = pk.vec(C.ptr);
  size_t o_gh = pk.vec(C.ghost);
  size_t o_w = pk.reals(C.w, p.dtype);
  size_t o_rot = pk.vec(C.rot);
  size_t o_cnt = pk.vec(C.cnt);
  size_t o_fg = pk.vec(C.fghost);
  size_t o_fw = pk.reals(C.fw, p.dtype);
  size_t o_frot = pk.vec(C.frot);
  void* dev = nullptr;
  HIP_CHECK(hipMalloc(&dev, pk.buf.size()));
  p.d_csc_dev = dev;
  HIP_CHECK(hipMemcpy(dev, pk.buf.data(), pk.buf.size(), hipMemcpyHostToDevice));
  char* b = static_cast<char*>(dev);
  p.d_csc_src = reinterpret_cast<const int64_t*>(b + o_src);
  p.d_csc_ptr = reinterpret_cast<const int64_t*>(b + o_ptr);
  p.d_csc_ghost = reinterpret_cast<const int64_t*>(b + o_gh);
  p.d_csc_w = b + o_w;
  p.d_csc_rot = reinterpret_cast<const int32_t*>(b + o_rot);
  p.d_adj_cnt = reinterpret_cast<const int32_t*>(b + o_cnt);
  p.d_adj_fg = reinterpret_cast<const int32_t*>(b + o_fg);
  p.d_adj_fw = b + o_fw;
  p.d_adj_frot = reinterpret_cast<const int8_t*>(b + o_frot);
  const AdjLdsHost& A = p.host.adj_lds;
  if (A.ok) {
    Packer q;
    size_t o_t = q.vec(A.tiles);
    size_t o_uc = q.vec(A.u_cell);
    size_t o_uk = q.vec(A.u_ctr);
    size_t o_ci = q.vec(A.ctr_init);
    size_t o_ct = q.vec(A.ctr_init);  // counters start at their reader counts
    size_t o_sl = q.vec(A.slot);
    size_t o_z = q.vec(A.zero_rows);
    void* dv = nullptr;
    HIP_CHECK(hipMalloc(&dv, q.buf.size()));
    p.d_al_dev = dv;
    HIP_CHECK(hipMemcpy(dv, q.buf.data(), q.buf.size(), hipMemcpyHostToDevice));
    char* c = static_cast<char*>(dv);
    p.d_al_tiles = reinterpret_cast<const AdjLdsTile*>(c + o_t);
    p.d_al_ucell = reinterpret_cast<const int32_t*>(c + o_uc);
    p.d_al_uctr = reinterpret_cast<const int32_t*>(c + o_uk);
    p.d_al_ctrinit = reinterpret_cast<const int32_t*>(c + o_ci);
    p.d_al_ctr = reinterpret_cast<int32_t*>(c + o_ct);
    p.d_al_slot = reinterpret_cast<const uint16_t*>(c + o_sl);
    p.d_al_zero = reinterpret_cast<const int32_t*>(c + o_z);
  }
  void* t = nullptr;
  size_t nt = std::max<size_t>(1, p.host.adj_tiles.size());
  HIP_CHECK(hipMalloc(&t, nt * sizeof(AdjTile)));
  if (!p.host.adj_tiles.empty())
    HIP_CHECK(hipMemcpy(t, p.host.adj_tiles.data(), p.host.adj_tiles.size() * sizeof(AdjTile), hipMemcpyHostToDevice));
  p.d_adj_tiles = static_cast<const AdjTile*>(t);
}

// While hbc_plan_kernels asks which kernels a call launches, the launch
// helpers below record each kernel instead of launching it (the same
// decisions as a real call, no GPU work).
static thread_local std::vector<const void*>* t_rec = nullptr;
#define HBC_LAUNCH(fn, ...)                                  \
  do {                                                       \
    if (t_rec)                                               \
      t_rec->push_back((const void*)(fn));                   \
    else                                                     \
      hipLaunchKernelGGL(fn, __VA_ARGS__);                   \
  } while (0)

template <typename T, int V, int U, int KX = 0>
static void launch_rows_vu(const PlanDesc& d, hipStream_t st, int grid, int blk, const RowTile* tiles, int nt, int z,
                           const DataDesc& dd) {
  const bool rb2 = rows_per_batch(1 << d.lpr_shift) == 2;
  // FP64 rows take the row-by-row fallback of non-sliding Lagrange batches
  // (C768 x 32 with b: 9.5-9.9 against 10.6-10.8 us); FP32 rows keep the
  // batched one (measured: 7.1-7.4 against 6.5-6.6 us row by row)
  constexpr int KS = sizeof(T) == 8 ? KM_SEQFB : 0;
  const dim3 g(grid + dd.grid), b(blk);
  if (d.general) {
    if (d.nt && rb2)
      HBC_LAUNCH((k_apply_rows<T, V, U, true, 2, 3 | KX | KS>), g, b, 0, st, d, tiles, nt, z, dd);
    else if (d.nt)
      HBC_LAUNCH((k_apply_rows<T, V, U, true, 4, 3 | KX | KS>), g, b, 0, st, d, tiles, nt, z, dd);
    else if (rb2)
      HBC_LAUNCH((k_apply_rows<T, V, U, false, 2, 3 | KX | KS>), g, b, 0, st, d, tiles, nt, z, dd);
    else
      HBC_LAUNCH((k_apply_rows<T, V, U, false, 4, 3 | KX | KS>), g, b, 0, st, d, tiles, nt, z, dd);
  } else {
    if (d.nt && rb2)
      HBC_LAUNCH((k_apply_rows<T, V, U, true, 2, 1 | KX | KS>), g, b, 0, st, d, tiles, nt, z, dd);
    else if (d.nt)
      HBC_LAUNCH((k_apply_rows<T, V, U, true, 4, 1 | KX | KS>), g, b, 0, st, d, tiles, nt, z, dd);
    else if (rb2)
      HBC_LAUNCH((k_apply_rows<T, V, U, false, 2, 1 | KX | KS>), g, b, 0, st, d, tiles, nt, z, dd);
    else
      HBC_LAUNCH((k_apply_rows<T, V, U, false, 4, 1 | KX | KS>), g, b, 0, st, d, tiles, nt, z, dd);
  }
}

// point-major row tiles: one instance per (vec, unroll) a plan can select
template <typename T>
static void launch_rows(const PlanDesc& d, hipStream_t st, int grid, int blk, const RowTile* tiles, int nt, int z,
                        const DataDesc& dd) {
  if (d.ua && dd.grid == 0) {
    launch_rows_vu<T, (sizeof(T) == 4 ? 4 : 2), 1, KM_UNAL>(d, st, grid, blk, tiles, nt, z, dd);
    return;
  }
  if (sizeof(T) == 4) {
    if (d.vec == 4)
      launch_rows_vu<T, (sizeof(T) == 4 ? 4 : 2), 1>(d, st, grid, blk, tiles, nt, z, dd);
    else if (d.vec == 2)
      d.unroll >= 2 ? launch_rows_vu<T, 2, 2>(d, st, grid, blk, tiles, nt, z, dd)
                    : launch_rows_vu<T, 2, 1>(d, st, grid, blk, tiles, nt, z, dd);
    else if (d.unroll >= 4)
      launch_rows_vu<T, 1, 4>(d, st, grid, blk, tiles, nt, z, dd);
    else
      d.unroll >= 2 ? launch_rows_vu<T, 1, 2>(d, st, grid, blk, tiles, nt, z, dd)
                    : launch_rows_vu<T, 1, 1>(d, st, grid, blk, tiles, nt, z, dd);
  } else {
    if (d.vec >= 2)
      launch_rows_vu<T, 2, 1>(d, st, grid, blk, tiles, nt, z, dd);
    else
      d.unroll >= 2 ? launch_rows_vu<T, 1, 2>(d, st, grid, blk, tiles, nt, z, dd)
                    : launch_rows_vu<T, 1, 1>(d, st, grid, blk, tiles, nt, z, dd);
  }
}

// Slices per workgroup of the wide-row kernel: up to 1 KiB of each row (the
// pipelined staging then has slices to overlap; measured best for 128- and
// 256-byte slices alike), while at least four workgroups per CU (256 CUs)
// remain.
static int wide_slices_per_wg(int ntiles, int nslices, int slice_bytes) {
  int spw = 1;
  while (spw < nslices && 2 * spw * slice_bytes <= 1024 &&
         (int64_t)ntiles * ((nslices + 2 * spw - 1) / (2 * spw)) >= 256 * 4)
    spw *= 2;
  return spw;
}

template <typename T, int V, int SB>
static void launch_wide(const Plan& p, const PlanDesc& d, hipStream_t st, bool zero_only, int nzero) {
  constexpr int S = SB / (int)sizeof(T);
  const int nslices = (int)((p.layout.inner + S - 1) / S);
  const int ntiles = (int)p.host.wtiles.size();
  const int spw = wide_slices_per_wg(ntiles, nslices, SB);
  const int nwide = ntiles * ((nslices + spw - 1) / spw);
  const int grid = nwide + nzero;
  const int ucap = p.host.w_maxu, ecap = (p.host.w_maxe + 1) & ~1;  // even: keeps the row starts 16-byte aligned
  const size_t lds = zero_only ? 0
                              : (size_t)ucap * SB + (size_t)ecap * sizeof(WideEnt<T>) +
                                    (size_t)(WIDE_ROWS + 1) * 4;
  const WideEnt<T>* went = static_cast<const WideEnt<T>*>(p.d_w_ent);
  if (d.nt)
    HBC_LAUNCH((k_apply_wide<T, V, SB, true>), dim3(grid), dim3(256), lds, st, d, p.d_wtiles, p.d_w_ucell,
                       p.d_w_row, p.d_w_rp, went, ucap, ecap, nslices, spw, zero_only ? 1 : 0, p.d_rtiles, nwide);
  else
    HBC_LAUNCH((k_apply_wide<T, V, SB, false>), dim3(grid), dim3(256), lds, st, d, p.d_wtiles, p.d_w_ucell,
                       p.d_w_row, p.d_w_rp, went, ucap, ecap, nslices, spw, zero_only ? 1 : 0, p.d_rtiles, nwide);
  HIP_CHECK(hipGetLastError());
}

// Sliding-window runs: one wavefront per (run, slice of 64 vectors), four
// per workgroup; nz zero-row tiles ride in extra workgroups.
template <typename T>
static void launch_win(const Plan& p, const PlanDesc& d, hipStream_t st, bool zero_only, int nz) {
  constexpr int V = 16 / (int)sizeof(T);
  const int64_t nvec = p.layout.inner / V;
  const int64_t nsl = (nvec + 63) / 64;
  const int64_t nitems = (int64_t)p.host.wruns.size() * nsl;
  if (nitems >= (int64_t(1) << 30)) fail(HBC_EUNSUPPORTED, "too many window runs for one launch");
  const int nwin = (int)((nitems + 3) / 4);
  const dim3 g((unsigned)(nwin + nz)), b(256);
  const int z = zero_only ? 1 : 0;
  const int rm = p.host.win_maxr;  // longest run: the smallest instance that holds it
#define HBC_WIN_O(RM, O, HB)                                                                                      \
  do {                                                                                                              \
    if (d.nt)                                                                                                       \
      HBC_LAUNCH((k_apply_win<T, V, true, RM, O, HB>), g, b, 0, st, d, p.d_wruns, (int)nitems, (int)nsl, z,  \
                         p.d_rtiles, nz);                                                                          \
    else                                                                                                            \
      HBC_LAUNCH((k_apply_win<T, V, false, RM, O, HB>), g, b, 0, st, d, p.d_wruns, (int)nitems, (int)nsl, z, \
                         p.d_rtiles, nz);                                                                          \
  } while (0)
#define HBC_WIN(RM)                         \
  do {                                      \
    if (p.tune.window_order)                \
      HBC_WIN_O(RM, true, false);           \
    else if (p.host.win_has_b)              \
      HBC_WIN_O(RM, false, true);           \
    else                                    \
      HBC_WIN_O(RM, false, false);          \
  } while (0)
  // one instance per run length the autotuner tries: every load slot of a
  // full run is used (a shorter run re-reads its last source row)
  if (rm <= 4)
    HBC_WIN(4);
  else if (rm <= 6)
    HBC_WIN(6);
  else if (rm <= 8)
    HBC_WIN(8);
  else if (rm <= 10)
    HBC_WIN(10);
  else if (rm <= 12)
    HBC_WIN(12);
  else
    HBC_WIN(16);
#undef HBC_WIN
#undef HBC_WIN_O
  HIP_CHECK(hipGetLastError());
}

template <typename T>
static void launch_apply_t(const Plan& p, const PlanDesc& d, hipStream_t st, bool zero_only) {
  const bool pm = p.layout.order == HBC_POINT_MAJOR;
  const int nt = (int)(pm ? p.host.rtiles.size() : p.host.tiles.size());
  const int grid = p.tune.persistent > 0 ? std::min(p.tune.persistent, nt) : nt;
  const int blk = p.tune.block;
  const int z = zero_only ? 1 : 0;
  DataDesc dd{p.d_dr_ptr, p.d_dr_col, p.d_dr_val, p.d_dr_scratch, 0, 0};
  if (!zero_only && p.stats.rows_data > 0 && !p.host.dc_ok) {
    // data rows gather into scratch in extra workgroups of this launch
    const int groups = blk / p.tune.lanes_per_row;
    dd.nrows = (int32_t)p.stats.rows_data;
    dd.grid = (int32_t)std::min<int64_t>((p.stats.rows_data + groups - 1) / groups, 4096);
  }
  // fold the row tiles into the first wide-row or window launch when they are
  // all zero rows without b (the corners of the cubed-sphere programs)
  const bool has_narrow = pm && !p.host.ntiles.empty(), has_wide = pm && !p.host.wtiles.empty();
  const bool has_win = pm && !p.host.wruns.empty();
  bool fold = (has_narrow || has_wide || has_win) && dd.grid == 0 && nt > 0;
  for (size_t k = 0; fold && k < p.host.rtiles.size(); ++k)
    fold = p.host.rtiles[k].kind == SEG_ZERO && !p.host.rtiles[k].has_b;
  if (has_narrow) {
    const int nn = (int)p.host.ntiles.size();
    HBC_LAUNCH((k_apply_narrow<T>), dim3(nn + (fold ? nt : 0)), dim3(256), 0, st, d, p.d_ntiles, z,
                       p.d_rtiles, nn);
    HIP_CHECK(hipGetLastError());
  }
  if (has_wide) {
    const int nz = fold && !has_narrow ? nt : 0;
    if constexpr (sizeof(T) == 8) {
      if (wide_slice_bytes(p) == 2 * WIDE_ROW_BYTES)
        launch_wide<T, 4, 2 * WIDE_ROW_BYTES>(p, d, st, zero_only, nz);
      else if (p.vec >= 2)
        launch_wide<T, 2, WIDE_ROW_BYTES>(p, d, st, zero_only, nz);
      else
        launch_wide<T, 1, WIDE_ROW_BYTES>(p, d, st, zero_only, nz);
    } else {
      if (p.vec == 4)
        launch_wide<T, 4, WIDE_ROW_BYTES>(p, d, st, zero_only, nz);
      else if (p.vec >= 2)
        launch_wide<T, 2, WIDE_ROW_BYTES>(p, d, st, zero_only, nz);
      else
        launch_wide<T, 1, WIDE_ROW_BYTES>(p, d, st, zero_only, nz);
    }
  }
  if (has_win) launch_win<T>(p, d, st, zero_only, fold && !has_narrow && !has_wide ? nt : 0);
  if (fold || grid + dd.grid == 0) return;
  if (!pm) {
    if (grid > 0) HBC_LAUNCH((k_apply_pm<T>), dim3(grid), dim3(blk), 0, st, d, p.d_tiles, nt, z);
  } else {
    launch_rows<T>(d, st, grid, blk, p.d_rtiles, nt, z, dd);
  }
  HIP_CHECK(hipGetLastError());
}

template <typename T, int V>
static void launch_data_scatter(const Plan& p, const PlanDesc& d, hipStream_t st) {
  const int n = (int)p.stats.rows_data;
  const int blk = p.tune.block;
  const int groups = blk >> d.lpr_shift;
  const int grid = (int)std::min<int64_t>((n + groups - 1) / groups, 4096);
  HBC_LAUNCH((k_data_scatter<T, V>), dim3(grid), dim3(blk), 0, st, d, p.d_dr_cell,
                     static_cast<const T*>(p.d_dr_scratch), n);
  HIP_CHECK(hipGetLastError());
}

template <typename T, int V>
static void launch_data_components(const Plan& p, const PlanDesc& d, hipStream_t st) {
  const int n = (int)p.host.dc_comp.size();
  const int blk = p.tune.block;
  const int groups = blk >> d.lpr_shift;
  const int grid = (int)std::min<int64_t>((n + groups - 1) / groups, 4096);
  if (d.nt)
    HBC_LAUNCH((k_data_components<T, V, true>), dim3(grid), dim3(blk), 0, st, d, p.d_dc_comp, p.d_dc_row_dst,
                       p.d_dc_row_ent, p.d_dc_row_n, p.d_dc_slot, static_cast<const T*>(p.d_dc_w), n);
  else
    HBC_LAUNCH((k_data_components<T, V, false>), dim3(grid), dim3(blk), 0, st, d, p.d_dc_comp, p.d_dc_row_dst,
                       p.d_dc_row_ent, p.d_dc_row_n, p.d_dc_slot, static_cast<const T*>(p.d_dc_w), n);
  HIP_CHECK(hipGetLastError());
}

template <typename T>
static void launch_data_scatter_v(const Plan& p, const PlanDesc& d, hipStream_t st) {
  if (p.host.dc_ok) {
    if (sizeof(T) == 4 && p.vec == 4)
      launch_data_components<T, (sizeof(T) == 4 ? 4 : 2)>(p, d, st);
    else if (p.vec >= 2)
      launch_data_components<T, 2>(p, d, st);
    else
      launch_data_components<T, 1>(p, d, st);
    return;
  }
  if (sizeof(T) == 4 && p.vec == 4)
    launch_data_scatter<T, (sizeof(T) == 4 ? 4 : 2)>(p, d, st);
  else if (p.vec >= 2)
    launch_data_scatter<T, 2>(p, d, st);
  else
    launch_data_scatter<T, 1>(p, d, st);
}

void device_apply(const Plan& p, void* field, void* stream, bool zero_only) {
  PlanDesc d = make_desc(p, field);
  const bool data_rows = !zero_only && p.stats.rows_data > 0;
  if (p.dtype == HBC_F64) {
    launch_apply_t<double>(p, d, S(stream), zero_only);
    if (data_rows) launch_data_scatter_v<double>(p, d, S(stream));
  } else {
    launch_apply_t<float>(p, d, S(stream), zero_only);
    if (data_rows) launch_data_scatter_v<float>(p, d, S(stream));
  }
}

// The LDS adjoint's own launch shape, whatever the forward's tuning: 256
// threads and few lanes per row, so that each row group walks few sources
// (its sources run one after another, a load then a store each).  Measured
// at C768 x 32 (rows of 8 and 16 vectors): 4 lanes per row beat 1, 2, 8 and
// 16 in FP64 and FP32.  Rows of fewer vectors take one lane per vector;
// longer rows a quarter of their vectors, at most 16 lanes (not measured).
template <int V>
static int adjoint_lds_lanes(const Plan& p) {
  const int64_t nvec = p.layout.inner / V;
  const int64_t want = nvec < 4 ? nvec : std::min<int64_t>(16, std::max<int64_t>(4, nvec / 4));
  int shift = 0;
  while ((int64_t(1) << shift) < want) ++shift;
  return shift;
}

template <typename T, int V>
static void launch_adjoint_lds(const Plan& p, const PlanDesc& d0, const AdjDesc& a, hipStream_t st, int32_t* ctr) {
  const AdjLdsHost& A = p.host.adj_lds;
  PlanDesc d = d0;
  d.lpr_shift = adjoint_lds_lanes<V>(p);
  AdjLdsDesc q{p.d_al_tiles, p.d_al_ucell, p.d_al_uctr, p.d_al_ctrinit, ctr ? ctr : p.d_al_ctr, p.d_al_slot,
               p.d_al_zero, (int32_t)A.tiles.size(), (int32_t)A.zero_rows.size()};
  const int grid = q.ntiles + (q.nzero + ADJ_ZERO_ROWS - 1) / ADJ_ZERO_ROWS;
  if (grid == 0) return;
  const size_t lds = (size_t)A.brows * p.layout.inner * sizeof(T);
  if (d.nt)
    HBC_LAUNCH((k_adjoint_lds<T, V, true>), dim3(grid), dim3(ADJ_LDS_BLOCK), lds, st, d, a, q);
  else
    HBC_LAUNCH((k_adjoint_lds<T, V, false>), dim3(grid), dim3(ADJ_LDS_BLOCK), lds, st, d, a, q);
  HIP_CHECK(hipGetLastError());
}

// Reader counters of the allocation-free adjoint: a file-scope device array
// (each GPU the library runs on holds its own copy until the process ends),
// shared by every such call on that GPU.
static __device__ __align__(256) int32_t scratch[ADJ_NOALLOC_COUNTERS];

// Device address of `scratch` on the current device, taken once per device
// with hipGetSymbolAddress (in host code the array's name is no device
// address).  No allocation: fixed slots for up to 64 devices.
static int32_t* scratch_address() {
  static std::mutex mu;
  static int32_t* addr[64] = {};
  int dev = 0;
  HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) fail(HBC_EUNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* a = nullptr;
    const hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !a) fail(HBC_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    addr[dev] = static_cast<int32_t*>(a);
  }
  return addr[dev];
}

__global__ __launch_bounds__(256) void k_copy_i32(int32_t* __restrict__ dst, const int32_t* __restrict__ src,
                                                  int n) {
  for (int i = blockIdx.x * 256 + (int)threadIdx.x; i < n; i += gridDim.x * 256) dst[i] = src[i];
}

// ctr: the reader counters to use (the plan's own, or the static scratch).
template <typename T>
static void launch_adjoint_t(const Plan& p, const PlanDesc& d, hipStream_t st, int32_t* ctr = nullptr) {
  AdjDesc a{p.d_csc_src, p.d_csc_ptr,  p.d_csc_ghost, p.d_csc_w,          p.d_csc_rot,
            p.d_adj_cnt, p.d_adj_fg, p.d_adj_fw,    p.d_adj_frot, p.host.csc.aw};
  if (p.host.adj_lds.ok && p.layout.order == HBC_POINT_MAJOR) {
    if (sizeof(T) == 4 && p.vec == 4)
      launch_adjoint_lds<T, (sizeof(T) == 4 ? 4 : 2)>(p, d, a, st, ctr);
    else if (p.vec >= 2)
      launch_adjoint_lds<T, 2>(p, d, a, st, ctr);
    else
      launch_adjoint_lds<T, 1>(p, d, a, st, ctr);
    return;
  }
  const int nt = (int)p.host.adj_tiles.size();
  if (nt > 0) {
    const int blk = p.tune.block;
    if (p.layout.order == HBC_PLANE_MAJOR)
      HBC_LAUNCH((k_adjoint<T, 1, true, false>), dim3(nt), dim3(blk), 0, st, d, a, p.d_adj_tiles, nt);
    else if (p.vec == 4 && d.nt)
      HBC_LAUNCH((k_adjoint<T, 4, false, true>), dim3(nt), dim3(blk), 0, st, d, a, p.d_adj_tiles, nt);
    else if (p.vec == 4)
      HBC_LAUNCH((k_adjoint<T, 4, false, false>), dim3(nt), dim3(blk), 0, st, d, a, p.d_adj_tiles, nt);
    else if (p.vec == 2 && d.nt)
      HBC_LAUNCH((k_adjoint<T, 2, false, true>), dim3(nt), dim3(blk), 0, st, d, a, p.d_adj_tiles, nt);
    else if (p.vec == 2)
      HBC_LAUNCH((k_adjoint<T, 2, false, false>), dim3(nt), dim3(blk), 0, st, d, a, p.d_adj_tiles, nt);
    else if (d.nt)
      HBC_LAUNCH((k_adjoint<T, 1, false, true>), dim3(nt), dim3(blk), 0, st, d, a, p.d_adj_tiles, nt);
    else
      HBC_LAUNCH((k_adjoint<T, 1, false, false>), dim3(nt), dim3(blk), 0, st, d, a, p.d_adj_tiles, nt);
    HIP_CHECK(hipGetLastError());
  }
  launch_apply_t<T>(p, d, st, true);  // covered ghost gradients := 0, after the gather
}

void device_adjoint(const Plan& p, void* grad, void* stream) {
  PlanDesc d = make_desc(p, grad);
  if (p.dtype == HBC_F64)
    launch_adjoint_t<double>(p, d, S(stream));
  else
    launch_adjoint_t<float>(p, d, S(stream));
}

std::vector<std::string> device_kernel_names(const Plan& p, int op) {
  std::vector<const void*> fns;
  t_rec = &fns;
  try {
    if (op == HBC_OP_ADJOINT)
      device_adjoint(p, nullptr, nullptr);
    else
      device_apply(p, nullptr, nullptr, false);
  } catch (...) {
    t_rec = nullptr;
    throw;
  }
  t_rec = nullptr;
  std::vector<std::string> out;
  for (const void* f : fns) {
    const char* nm = hipKernelNameRefByPtr(f, nullptr);
    if (!nm) fail(HBC_EHIP, "hipKernelNameRefByPtr gave no name");
    int status = 0;
    char* dm = abi::__cxa_demangle(nm, nullptr, nullptr, &status);
    out.emplace_back(status == 0 && dm ? dm : nm);
    std::free(dm);
  }
  return out;
}

void device_adjoint_noalloc(const Plan& p, void* grad, void* stream) {
  PlanDesc d = make_desc(p, grad);
  int32_t* ctr = nullptr;
  if (p.host.adj_lds.ok && p.layout.order == HBC_POINT_MAJOR) {
    const size_t n = p.host.adj_lds.ctr_init.size();
    if (n > (size_t)ADJ_NOALLOC_COUNTERS)
      fail(HBC_EINVAL, "the plan needs " + std::to_string(n) + " reader counters; the allocation-free adjoint holds " +
                           std::to_string(ADJ_NOALLOC_COUNTERS));
    ctr = scratch_address();
    if (n > 0) {
      // the array keeps whatever the last call on this GPU left: start every
      // counter at its reader count (a copy kernel, so the call can be captured)
      const int grid = (int)std::min<size_t>((n + 255) / 256, 1024);
      hipLaunchKernelGGL(k_copy_i32, dim3(grid), dim3(256), 0, S(stream), ctr, p.d_al_ctrinit, (int)n);
      HIP_CHECK(hipGetLastError());
    }
  }
  if (p.dtype == HBC_F64)
    launch_adjoint_t<double>(p, d, S(stream), ctr);
  else
    launch_adjoint_t<float>(p, d, S(stream), ctr);
}

void device_stencil27(Plan& p, const void* x, void* y, void* stream, bool fused, void* xghost) {
  if (!p.st_ok) fail(HBC_EUNSUPPORTED, p.st_reason.empty() ? "plan not usable by the 27-point consumer" : p.st_reason);
  if (fused && (!p.st_fused || !p.d_st_info))
    fail(HBC_EUNSUPPORTED, p.st_fused_reason.empty() ? "plan not usable by the fused 27-point consumer" : p.st_fused_reason);
  StDesc st;
  st.nblk = p.st_nblocks;
  st.nz = (int32_t)p.st_n[0];
  st.ny = (int32_t)p.st_n[1];
  st.nx = (int32_t)p.st_n[2];
  st.sy = st.nx + 2;
  st.sz = (int64_t)(st.ny + 2) * st.sy;
  st.bcells = (int64_t)(st.nz + 2) * st.sz;
  st.info = p.d_st_info;
  const int ntx = (st.nx + ST_TX - 1) / ST_TX, nty = (st.ny + ST_TY - 1) / ST_TY, nzc = (st.nz + ST_ZC - 1) / ST_ZC;
  const int64_t grid = (int64_t)ntx * nty * nzc * st.nblk;
  if (grid >= (int64_t(1) << 31)) fail(HBC_EUNSUPPORTED, "grid too large for the 27-point consumer");
  // each workgroup's x and y ranges are buffer resources addressed in 32 bits
  const int64_t esz = p.dtype == HBC_F64 ? 8 : 4;
  if ((int64_t)(ST_ZC + 2) * st.sz * esz >= (int64_t)BUF_OOB || (int64_t)ST_ZC * st.ny * st.nx * esz >= (int64_t)BUF_OOB)
    fail(HBC_EUNSUPPORTED, "blocks too large for the 27-point consumer (32-plane chunks of 2 GiB or more)");
  hipStream_t s = S(stream);
  const dim3 g((unsigned)grid), blk(256);
  if (grid == 0) return;
  auto go = [&](auto tag) {
    using T = decltype(tag);
    const T* xt = static_cast<const T*>(x);
    T* yt = static_cast<T*>(y);
    if (!fused)
      hipLaunchKernelGGL((k_stencil27<T, false, false>), g, blk, 0, s, xt, nullptr, yt, st);
    else if (xghost)
      hipLaunchKernelGGL((k_stencil27<T, true, true>), g, blk, 0, s, xt, static_cast<T*>(xghost), yt, st);
    else
      hipLaunchKernelGGL((k_stencil27<T, true, false>), g, blk, 0, s, xt, nullptr, yt, st);
  };
  if (p.dtype == HBC_F64)
    go(double{});
  else
    go(float{});
  HIP_CHECK(hipGetLastError());
}

void device_cs_weights(int64_t N, int64_t h, int32_t* base, double* w, void* stream) {
  if (N * h >= (int64_t(1) << 30)) fail(HBC_EUNSUPPORTED, "grid too large");
  const int n = (int)(N * h);
  hipLaunchKernelGGL(k_cs_weights, dim3((n + 255) / 256), dim3(256), 0, S(stream), (int)N, (int)h, base, w);
  HIP_CHECK(hipGetLastError());
}

// ---- consumer tables and launch -------------------------------------------------------
struct ConsDev {
  void* dev = nullptr;
  const int32_t* delta = nullptr;
  const void* w = nullptr;
  const CTile* tiles_all = nullptr;
  const CTile* tiles_int = nullptr;
  const int32_t* brow_y = nullptr;
  const int32_t* bptr = nullptr;
  const int32_t* bcol = nullptr;
  const void* bw = nullptr;
  const int8_t* brot = nullptr;
  const int32_t* bconst_row = nullptr;
  const void* bconst = nullptr;
  const int32_t* line_delta = nullptr;
  const void* line_w = nullptr;
};

void* device_consumer_upload(const Plan& p, const ConsumerHost& C) {
  Packer pk;
  const size_t o_dl = pk.vec(C.delta), o_w = pk.reals(C.w, p.dtype), o_ta = pk.vec(C.tiles_all),
               o_ti = pk.vec(C.tiles_int), o_by = pk.vec(C.brow_y), o_bp = pk.vec(C.bptr), o_bc = pk.vec(C.bcol),
               o_bw = pk.reals(C.bw, p.dtype), o_br = pk.vec(C.brot), o_bk = pk.vec(C.bconst_row),
               o_bv = pk.reals(C.bconst, p.dtype), o_ld = pk.vec(C.line_delta), o_lw = pk.reals(C.line_w, p.dtype);
  auto* cd = new ConsDev;
  void* dev = nullptr;
  const hipError_t e = hipMalloc(&dev, pk.buf.size());
  if (e != hipSuccess) {
    delete cd;
    fail(e == hipErrorOutOfMemory ? HBC_ENOMEM : HBC_EHIP, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  cd->dev = dev;
  const hipError_t e2 = hipMemcpy(dev, pk.buf.data(), pk.buf.size(), hipMemcpyHostToDevice);
  if (e2 != hipSuccess) {
    (void)hipFree(dev);
    delete cd;
    fail(HBC_EHIP, std::string("hipMemcpy: ") + hipGetErrorString(e2));
  }
  char* b = static_cast<char*>(dev);
  cd->delta = reinterpret_cast<const int32_t*>(b + o_dl);
  cd->w = b + o_w;
  cd->tiles_all = reinterpret_cast<const CTile*>(b + o_ta);
  cd->tiles_int = reinterpret_cast<const CTile*>(b + o_ti);
  cd->brow_y = reinterpret_cast<const int32_t*>(b + o_by);
  cd->bptr = reinterpret_cast<const int32_t*>(b + o_bp);
  cd->bcol = reinterpret_cast<const int32_t*>(b + o_bc);
  cd->bw = b + o_bw;
  cd->brot = reinterpret_cast<const int8_t*>(b + o_br);
  cd->bconst_row = reinterpret_cast<const int32_t*>(b + o_bk);
  cd->bconst = b + o_bv;
  cd->line_delta = reinterpret_cast<const int32_t*>(b + o_ld);
  cd->line_w = b + o_lw;
  return cd;
}

void device_consumer_free(void* h) {
  auto* cd = static_cast<ConsDev*>(h);
  if (!cd) return;
  if (cd->dev) (void)hipFree(cd->dev);
  delete cd;
}

template <typename T, int V, int WALK>
static void launch_consumer_walk(bool nt, dim3 g, dim3 b, hipStream_t st, const PlanDesc& d, const ConsDesc& c) {
  if (nt)
    hipLaunchKernelGGL((k_consumer<T, V, true, WALK>), g, b, 0, st, d, c);
  else
    hipLaunchKernelGGL((k_consumer<T, V, false, WALK>), g, b, 0, st, d, c);
}

template <typename T, int V>
static void launch_consumer(bool nt, int nlines, dim3 g, dim3 b, hipStream_t st, const PlanDesc& d,
                            const ConsDesc& c) {
  // one pass of a row group per cell: the line walk, else the pipelined walk
  // for at most 8 offsets
  const bool one_pass = d.inner / V <= (int64_t(1) << d.lpr_shift);
  static_assert(CONS_MAXLINES == 3, "one line-walk instance per line count");
  if (one_pass && nlines == 1)
    launch_consumer_walk<T, V, 11>(nt, g, b, st, d, c);
  else if (one_pass && nlines == 2)
    launch_consumer_walk<T, V, 12>(nt, g, b, st, d, c);
  else if (one_pass && nlines == 3)
    launch_consumer_walk<T, V, 13>(nt, g, b, st, d, c);
  else if (one_pass && c.noff <= 8)
    launch_consumer_walk<T, V, 1>(nt, g, b, st, d, c);
  else
    launch_consumer_walk<T, V, 0>(nt, g, b, st, d, c);
}

void device_consumer_apply(const Plan& p, const ConsumerHost& C, void* h, const void* x, void* y, bool fused,
                           void* stream) {
  const auto* cd = static_cast<const ConsDev*>(h);
  PlanDesc d = make_desc(p, const_cast<void*>(x));
  ConsDesc c{};
  c.delta = cd->delta;
  c.w = cd->w;
  c.noff = C.noff;
  c.tiles = fused ? cd->tiles_int : cd->tiles_all;
  c.ntiles = (int32_t)(fused ? C.tiles_int.size() : C.tiles_all.size());
  c.brow_y = cd->brow_y;
  c.bptr = cd->bptr;
  c.bcol = cd->bcol;
  c.bw = cd->bw;
  c.brot = cd->brot;
  c.bconst_row = cd->bconst_row;
  c.bconst = cd->bconst;
  c.nbrow = fused ? (int32_t)C.brow_y.size() : 0;
  c.tile_rows = std::max(1, C.tile_rows);
  c.y = y;
  c.line_delta = cd->line_delta;
  c.line_w = cd->line_w;
  c.line_mask = C.line_mask;
  const int64_t nbt = (c.nbrow + c.tile_rows - 1) / c.tile_rows;
  const int64_t grid = (int64_t)c.ntiles + nbt;
  if (grid >= (int64_t(1) << 31)) fail(HBC_EUNSUPPORTED, "consumer grid too large");
  if (grid == 0) return;
  const dim3 g((unsigned)grid), blk(256);
  hipStream_t st = S(stream);
  if (p.dtype == HBC_F64) {
    if (p.vec >= 2)
      launch_consumer<double, 2>(d.nt != 0, C.nlines, g, blk, st, d, c);
    else
      launch_consumer<double, 1>(d.nt != 0, C.nlines, g, blk, st, d, c);
  } else {
    if (p.vec == 4)
      launch_consumer<float, 4>(d.nt != 0, C.nlines, g, blk, st, d, c);
    else if (p.vec == 2)
      launch_consumer<float, 2>(d.nt != 0, C.nlines, g, blk, st, d, c);
    else
      launch_consumer<float, 1>(d.nt != 0, C.nlines, g, blk, st, d, c);
  }
  HIP_CHECK(hipGetLastError());
}

// ---- timing of plain applies under a captured graph ------------------------------------
namespace {
struct OwnedStream {
  hipStream_t s = nullptr;
  bool owned = false;
  explicit OwnedStream(void* given) {
    if (given) {
      s = S(given);
    } else {
      HIP_CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      owned = true;
    }
  }
  ~OwnedStream() {
    if (owned) (void)hipStreamDestroy(s);
  }
};
}  // namespace

double device_time_apply(const Plan& p, void* const* fields, int nfields, int reps, void* stream) {
  OwnedStream os(stream);
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  HIP_CHECK(hipStreamBeginCapture(os.s, hipStreamCaptureModeThreadLocal));
  try {
    for (int r = 0; r < reps; ++r) device_apply(p, fields[r % nfields], os.s, false);
  } catch (...) {
    (void)hipStreamEndCapture(os.s, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  HIP_CHECK(hipStreamEndCapture(os.s, &graph));
  HIP_CHECK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  hipEvent_t e0, e1;
  HIP_CHECK(hipEventCreate(&e0));
  HIP_CHECK(hipEventCreate(&e1));
  HIP_CHECK(hipGraphLaunch(exec, os.s));  // warm
  HIP_CHECK(hipEventRecord(e0, os.s));
  HIP_CHECK(hipGraphLaunch(exec, os.s));
  HIP_CHECK(hipEventRecord(e1, os.s));
  HIP_CHECK(hipEventSynchronize(e1));
  float ms = 0;
  HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipGraphExecDestroy(exec);
  (void)hipGraphDestroy(graph);
  return (double)ms / reps;
}

struct ApplyGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const Plan* plan = nullptr;
  uint64_t gen = 0;  // the plan's tile generation at capture
};

void* device_graph_create(const Plan& p, int op, void* const* fields, int nfields, int reps, void* stream) {
  if (!stream) fail(HBC_EINVAL, "graph capture needs a stream");
  auto* g = new ApplyGraph;
  g->plan = &p;
  g->gen = p.tile_gen;
  hipStream_t s = S(stream);
  hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    delete g;
    fail(HBC_EHIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
  }
  try {
    for (int r = 0; r < reps; ++r) {
      if (op == HBC_OP_ADJOINT)
        device_adjoint(p, fields[r % nfields], stream);
      else
        device_apply(p, fields[r % nfields], stream, false);
    }
  } catch (...) {
    (void)hipStreamEndCapture(s, &g->graph);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    throw;
  }
  e = hipStreamEndCapture(s, &g->graph);
  if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    device_graph_destroy(g);
    fail(HBC_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
  }
  return g;
}

void device_graph_launch(void* gp, void* stream) {
  auto* g = static_cast<ApplyGraph*>(gp);
  if (g->plan->tile_gen != g->gen)
    fail(HBC_EINVAL, "the plan's launch shape changed after this graph was captured (tuning rebuilds the tile "
                     "tables the graph points at); capture it again");
  HIP_CHECK(hipGraphLaunch(g->exec, S(stream)));
}

void device_graph_destroy(void* gp) {
  auto* g = static_cast<ApplyGraph*>(gp);
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

// ---- batched persistent apply ------------------------------------------------------------
struct Batch {
  std::vector<Plan*> plans;
  int dtype = HBC_F64;
  hbc_tune tune{};
  std::vector<PlanDesc> descs;
  PlanDesc* d_descs = nullptr;
  std::vector<RowTile> tiles;
  RowTile* d_tiles = nullptr;
  bool bound = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hbc_stats stats{};
};

// Rows per batch of a row group in the batch kernel (rt_tile_any's choice
// for the plan's vector width and unroll).
static int batch_rows_per_batch(const PlanDesc& d, int dtype) {
  if (d.ua) return 4;
  if (dtype == HBC_F32) {
    if (d.vec == 4) return 4;
    if (d.vec == 2) return d.unroll >= 2 ? 2 : 4;
    return d.unroll >= 2 ? 2 : 4;
  }
  if (d.vec >= 2) return 4;
  return d.unroll >= 2 ? 2 : 4;
}

static void batch_tiles(Batch* b) {
  // per plan: rows per tile so that a tile holds about tune.rows_per_tile inner
  // values; rows_per_tile = 0 gives every row group one batch of rows (all
  // loads of a workgroup issued before its first store)
  std::vector<std::vector<RowTile>> per(b->plans.size());
  for (size_t k = 0; k < b->plans.size(); ++k) {
    const Plan& p = *b->plans[k];
    const int64_t I = p.layout.inner;
    int lpr = p.tune.lanes_per_row;
    if (b->tune.lanes_per_row > 0) lpr = std::min(lpr, b->tune.lanes_per_row);
    b->descs[k].lpr_shift = ilog2(lpr);
    b->descs[k].chunked = lpr >= CHUNK_LPR ? 1 : 0;
    const int64_t rp = std::max<int64_t>(1, b->tune.block / lpr);
    int64_t rpt = std::max<int64_t>(1, (int64_t)b->tune.rows_per_tile / I);
    rpt = ((rpt + rp - 1) / rp) * rp;
    if (b->tune.rows_per_tile == 0) rpt = rp * batch_rows_per_batch(b->descs[k], b->dtype);
    rpt = std::min<int64_t>(rpt, 1 << 20);
    for (size_t s = 0; s < p.host.segs.size(); ++s) {
      const DevSeg& sg = p.host.segs[s];
      for (int64_t r0 = 0; r0 < sg.nrows; r0 += rpt) {
        RowTile rt{};
        rt.kind = sg.kind;
        rt.rot = sg.rot;
        rt.flags = sg.flags;
        rt.width = sg.width;
        rt.row_begin = sg.row_base + r0;
        rt.tab = sg.kind == SEG_ELL ? sg.tab + r0 * sg.width : sg.tab + r0;
        rt.brow = sg.brow + r0 * sg.b_inner;
        rt.w = sg.w;
        rt.nrows = (int32_t)std::min<int64_t>(rpt, sg.nrows - r0);
        rt.has_b = sg.has_b;
        rt.b_inner = sg.b_inner;
        rt.pad_ = (int32_t)k;  // plan index
        per[k].push_back(rt);
      }
    }
  }
  // interleave plans round-robin so that every part of the launch mixes grids
  b->tiles.clear();
  size_t more = 1;
  for (size_t i = 0; more; ++i) {
    more = 0;
    for (auto& v : per)
      if (i < v.size()) {
        b->tiles.push_back(v[i]);
        more = 1;
      }
  }
  // the captured graph (if any) points at the old tile table
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  if (b->d_tiles) HIP_CHECK(hipFree(b->d_tiles));
  b->d_tiles = nullptr;
  HIP_CHECK(hipMalloc(&b->d_tiles, std::max<size_t>(1, b->tiles.size()) * sizeof(RowTile)));
  if (!b->tiles.empty())
    HIP_CHECK(hipMemcpy(b->d_tiles, b->tiles.data(), b->tiles.size() * sizeof(RowTile), hipMemcpyHostToDevice));
  b->stats.tiles = (int64_t)b->tiles.size();
  if (b->bound) device_batch_bind(b, nullptr);
}

Batch* device_batch_create(Plan* const* plans, int n) {
  Batch* b = new Batch;
  try {
    b->plans.assign(plans, plans + n);
    b->dtype = plans[0]->dtype;
    b->descs.resize(n);
    std::memset(&b->stats, 0, sizeof(b->stats));
    for (int k = 0; k < n; ++k) {
      b->descs[k] = make_desc(*plans[k], nullptr);
      const hbc_stats& s = plans[k]->stats;
      b->stats.ghost_cells += s.ghost_cells;
      b->stats.rows_covered += s.rows_covered;
      b->stats.rows_uncovered += s.rows_uncovered;
      b->stats.rows_zero += s.rows_zero;
      b->stats.rows_map += s.rows_map;
      b->stats.rows_ell += s.rows_ell;
      b->stats.rows_csr += s.rows_csr;
      b->stats.rows_vector_only += s.rows_vector_only;
      b->stats.rows_with_b += s.rows_with_b;
      b->stats.nnz += s.nnz;
      b->stats.unique_sources += s.unique_sources;
      b->stats.segments += s.segments;
      b->stats.ghost_values += s.ghost_values;
      b->stats.alg_bytes += s.alg_bytes;
      b->stats.alg_bytes_adjoint += s.alg_bytes_adjoint;
      b->stats.table_bytes += (int64_t)plans[k]->dev_bytes;
    }
    HIP_CHECK(hipMalloc(&b->d_descs, n * sizeof(PlanDesc)));
    b->tune.block = 256;
    b->tune.lanes_per_row = 0;
    b->tune.rows_per_tile = 8192;
    int dev = 0, ncu = 256;
    HIP_CHECK(hipGetDevice(&dev));
    HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    b->tune.persistent = 4 * ncu;
    batch_tiles(b);
  } catch (...) {
    device_batch_destroy(b);
    throw;
  }
  return b;
}

void device_batch_destroy(Batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->d_descs) (void)hipFree(b->d_descs);
  if (b->d_tiles) (void)hipFree(b->d_tiles);
  delete b;
}

void device_update_b(Plan& p, int64_t first, int64_t last, void* stream) {
  if (last <= first) return;
  const size_t es = p.dtype == HBC_F64 ? 8 : 4, n = (size_t)(last - first);
  std::vector<unsigned char> buf(n * es);
  if (p.dtype == HBC_F64) {
    std::memcpy(buf.data(), p.host.bval.data() + first, n * es);
  } else {
    float* f = reinterpret_cast<float*>(buf.data());
    for (size_t k = 0; k < n; ++k) f[k] = (float)p.host.bval[first + k];  // rounded as at plan creation
  }
  // ordered after earlier work on the stream; the call returns once the copy is done
  unsigned char* dst = static_cast<unsigned char*>(const_cast<void*>(p.d_bval)) + (size_t)first * es;
  HIP_CHECK(hipMemcpyAsync(dst, buf.data(), n * es, hipMemcpyHostToDevice, S(stream)));
  HIP_CHECK(hipStreamSynchronize(S(stream)));
}

void device_batch_bind(Batch* b, void* const* fields) {
  if (fields)
    for (size_t k = 0; k < b->plans.size(); ++k) {
      if (!fields[k] || ((uintptr_t)fields[k] & 15)) fail(HBC_EINVAL, "batch field NULL or not 16-byte aligned");
      b->descs[k].field = fields[k];
    }
  HIP_CHECK(hipMemcpy(b->d_descs, b->descs.data(), b->descs.size() * sizeof(PlanDesc), hipMemcpyHostToDevice));
  b->bound = true;
}

void device_batch_apply(Batch* b, void* stream) {
  if (!b->bound) fail(HBC_EINVAL, "bind fields before applying a batch");
  const int nt = (int)b->tiles.size();
  if (nt == 0) return;
  const int grid = b->tune.persistent > 0 ? std::min(b->tune.persistent, nt) : nt;
  bool gen = false;  // any general ELL/CSR rows among the tiles
  for (const RowTile& t : b->tiles)
    if (t.kind == SEG_CSR || (t.kind == SEG_ELL && (t.width != 4 || (t.flags & SEGF_ELL_PADDED)))) gen = true;
  const dim3 g(grid), blk(b->tune.block);
  if (b->dtype == HBC_F64) {
    if (gen)
      hipLaunchKernelGGL((k_batch<double, 3 | KM_SEQFB>), g, blk, 0, S(stream), b->d_descs, b->d_tiles, nt);
    else
      hipLaunchKernelGGL((k_batch<double, 1 | KM_SEQFB>), g, blk, 0, S(stream), b->d_descs, b->d_tiles, nt);
  } else {
    if (gen)
      hipLaunchKernelGGL((k_batch<float, 3 | KM_SEQFB>), g, blk, 0, S(stream), b->d_descs, b->d_tiles, nt);
    else
      hipLaunchKernelGGL((k_batch<float, 1 | KM_SEQFB>), g, blk, 0, S(stream), b->d_descs, b->d_tiles, nt);
  }
  HIP_CHECK(hipGetLastError());
}

void device_batch_capture(Batch* b, void* stream) {
  if (!stream) fail(HBC_EINVAL, "graph capture needs a stream");
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  HIP_CHECK(hipStreamBeginCapture(S(stream), hipStreamCaptureModeThreadLocal));
  try {
    device_batch_apply(b, stream);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(S(stream), &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  HIP_CHECK(hipStreamEndCapture(S(stream), &b->graph));
  HIP_CHECK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
}

void device_batch_launch_graph(Batch* b, void* stream) {
  if (!b->exec) fail(HBC_EINVAL, "no captured graph");
  HIP_CHECK(hipGraphLaunch(b->exec, S(stream)));
}

hbc_tune device_batch_get_tune(const Batch* b) { return b->tune; }

void device_batch_set_tune(Batch* b, const hbc_tune& t) {
  if (t.block < 64 || t.block > 256 || t.block % 64) fail(HBC_EINVAL, "block must be 64, 128, 192 or 256");
  if (t.lanes_per_row < 0 || (t.lanes_per_row & (t.lanes_per_row - 1))) fail(HBC_EINVAL, "lanes_per_row: 0 or a power of two");
  if (t.rows_per_tile < 0 || t.persistent < 0) fail(HBC_EINVAL, "bad tile size or persistent count");
  b->tune = t;
  batch_tiles(b);
}

void device_batch_stats(const Batch* b, hbc_stats* out) { *out = b->stats; }

// Generation of the kernels' performance, part of every autotune cache key:
// a choice stored by a build whose kernels time differently is not reused
// (bumped with such changes; 2: window loads at raised priority, where runs
// of 4 turned from the fastest to among the slowest).
constexpr int TUNE_CACHE_GEN = 2;

static std::string batch_key(const Batch* b) {
  int dev = 0;
  hipDeviceProp_t prop;
  HIP_CHECK(hipGetDevice(&dev));
  HIP_CHECK(hipGetDeviceProperties(&prop, dev));
  std::ostringstream k;
  k << prop.gcnArchName << "|g" << TUNE_CACHE_GEN << "|" << (b->dtype == HBC_F64 ? "f64" : "f32") << "|point|"
    << b->plans.size() << "|"
    << b->stats.ghost_values << "|" << b->stats.rows_covered;
  std::string s = k.str();
  for (char& c : s)
    if (c == '"' || c == '\\') c = '_';
  return s;
}

static double time_batch(Batch* b, hipStream_t s, int reps) {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  for (int r = 0; r < reps; ++r) device_batch_apply(b, s);
  HIP_CHECK(hipStreamEndCapture(s, &graph));
  HIP_CHECK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  hipEvent_t e0, e1;
  HIP_CHECK(hipEventCreate(&e0));
  HIP_CHECK(hipEventCreate(&e1));
  HIP_CHECK(hipGraphLaunch(exec, s));
  HIP_CHECK(hipEventRecord(e0, s));
  HIP_CHECK(hipGraphLaunch(exec, s));
  HIP_CHECK(hipEventRecord(e1, s));
  HIP_CHECK(hipEventSynchronize(e1));
  float ms = 0;
  HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipGraphExecDestroy(exec);
  (void)hipGraphDestroy(graph);
  return (double)ms / reps;
}

// ---- plan autotuner ------------------------------------------------------------------------
static std::string plan_key(const Plan& p) {
  int dev = 0;
  hipDeviceProp_t prop;
  HIP_CHECK(hipGetDevice(&dev));
  HIP_CHECK(hipGetDeviceProperties(&prop, dev));
  std::ostringstream k;
  k << prop.gcnArchName << "|g" << TUNE_CACHE_GEN << "|plan|" << (p.dtype == HBC_F64 ? "f64" : "f32") << "|"
    << (p.layout.order == HBC_POINT_MAJOR ? "point" : "plane") << "|" << p.layout.inner << "|" << p.vec << "|"
    << p.stats.rows_covered << "|" << p.stats.segments << "|" << p.stats.nnz << "|" << p.stats.rows_data << "|w"
    << (windows_possible(p) ? 1 : 0);
  std::string s = k.str();
  for (char& c : s)
    if (c == '"' || c == '\\') c = '_';
  return s;
}

// Try launch shapes on the given fields (cycled, so the timing sees cold
// caches when the fields are many), keep the fastest.  Results do not depend
// on the shape; only the tile table changes.
double device_plan_autotune(Plan& p, void* const* fields, int nfields, const char* cache_path, void* stream) {
  const std::string key = plan_key(p);
  const int reps = std::max(2 * nfields, 12);
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      if (line.find("\"key\": \"" + key + "\"") == std::string::npos) continue;
      hbc_tune t{};
      double ms = 0;
      if (std::sscanf(line.c_str() + line.find("\"block\""),
                      "\"block\": %d, \"lanes_per_row\": %d, \"rows_per_tile\": %d, \"persistent\": %d, "
                      "\"window_order\": %d, \"ms\": %lf",
                      &t.block, &t.lanes_per_row, &t.rows_per_tile, &t.persistent, &t.window_order, &ms) == 6) {
        build_tiles(p, t);
        device_upload_tiles(p);
        return device_time_apply(p, fields, nfields, reps, stream);
      }
    }
  }
  int dev = 0, ncu = 256;
  HIP_CHECK(hipGetDevice(&dev));
  HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const hbc_tune def = default_tune(p);
  std::vector<hbc_tune> cand;
  if (p.stats.rows_window > 0) {
    // window plans: the run length (a run's three extra cells against the
    // number of wavefronts in flight) and the order of loads and stores
    for (int r : {4, 6, 8, 10, 12, 16})
      for (int o : {0, 1}) {
        hbc_tune t = def;
        t.rows_per_tile = r;
        t.window_order = o;
        cand.push_back(t);
      }
  } else {
    for (int bl : {128, 256})
      for (int lf : {1, 2}) {
        const int lpr = std::max(1, std::min(bl, def.lanes_per_row / lf));
        const int rp = bl / lpr;
        for (int m : {1, 2, 4, 8})
          for (int pf : {0, 4}) cand.push_back(hbc_tune{bl, lpr, rp * m, pf * ncu});
      }
  }
  cand.push_back(def);
  hbc_tune best = def;
  double best_ms = 1e30;
  for (const hbc_tune& t : cand) {
    build_tiles(p, t);
    device_upload_tiles(p);
    const double ms = device_time_apply(p, fields, nfields, reps, stream);
    if (ms < best_ms) {
      best_ms = ms;
      best = t;
    }
  }
  build_tiles(p, best);
  device_upload_tiles(p);
  best_ms = device_time_apply(p, fields, nfields, reps, stream);
  if (cache_path) {
    std::ofstream out(cache_path, std::ios::app);
    out << "{\"key\": \"" << key << "\", \"block\": " << best.block << ", \"lanes_per_row\": " << best.lanes_per_row
        << ", \"rows_per_tile\": " << best.rows_per_tile << ", \"persistent\": " << best.persistent
        << ", \"window_order\": " << best.window_order << ", \"ms\": " << best_ms << "}\n";
  }
  return best_ms;
}

double device_batch_autotune(Batch* b, const char* cache_path, void* stream) {
  if (!b->bound) fail(HBC_EINVAL, "bind fields before tuning a batch");
  OwnedStream os(stream);
  const std::string key = batch_key(b);
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      if (line.find("\"key\": \"" + key + "\"") == std::string::npos) continue;
      hbc_tune t{};
      double ms = 0;
      if (std::sscanf(line.c_str() + line.find("\"block\""), "\"block\": %d, \"lanes_per_row\": %d, \"rows_per_tile\": %d, \"persistent\": %d, \"ms\": %lf",
                      &t.block, &t.lanes_per_row, &t.rows_per_tile, &t.persistent, &ms) == 5) {
        device_batch_set_tune(b, t);
        return time_batch(b, os.s, 5);
      }
    }
  }
  int dev = 0, ncu = 256;
  HIP_CHECK(hipGetDevice(&dev));
  HIP_CHECK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const hbc_tune start = b->tune;
  hbc_tune best = start;
  double best_ms = 1e30;
  const int blocks[] = {128, 256};
  const int elems[] = {0, 4096, 8192, 16384, 32768};  // 0: one batch of rows per row group
  const int pers[] = {0, 2, 4, 8};
  const int lprs[] = {0, 32};
  for (int bl : blocks)
    for (int el : elems)
      for (int pf : pers)
        for (int lp : lprs) {
          hbc_tune t{bl, lp, el, pf * ncu};
          device_batch_set_tune(b, t);
          double ms = time_batch(b, os.s, 3);
          if (ms < best_ms) {
            best_ms = ms;
            best = t;
          }
        }
  device_batch_set_tune(b, best);
  best_ms = time_batch(b, os.s, 5);
  if (cache_path) {
    std::ofstream out(cache_path, std::ios::app);
    out << "{\"key\": \"" << key << "\", \"block\": " << best.block << ", \"lanes_per_row\": " << best.lanes_per_row
        << ", \"rows_per_tile\": " << best.rows_per_tile << ", \"persistent\": " << best.persistent
        << ", \"ms\": " << best_ms << "}\n";
  }
  return best_ms;
}

}  // namespace hbc
