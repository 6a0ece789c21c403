// Internal structures shared by the host plan compiler and the HIP launchers.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hbc.h"

namespace hbc {

// ---- errors -----------------------------------------------------------------
struct Error {
  int code;
  std::string msg;
};
void set_error(const std::string& msg);
[[noreturn]] void fail(int code, const std::string& msg);

// ---- boxes ------------------------------------------------------------------
struct Box {
  int nd = 0;
  int64_t lo[HBC_MAX_DIM] = {0};
  int64_t hi[HBC_MAX_DIM] = {0};
  int64_t extent(int d) const { return hi[d] - lo[d]; }
  int64_t count() const {
    int64_t n = 1;
    for (int d = 0; d < nd; ++d) n *= (hi[d] > lo[d] ? hi[d] - lo[d] : 0);
    return n;
  }
  bool empty() const { return count() == 0; }
  bool contains(const int64_t* c) const {
    for (int d = 0; d < nd; ++d)
      if (c[d] < lo[d] || c[d] >= hi[d]) return false;
    return true;
  }
  bool contains(const Box& b) const {
    for (int d = 0; d < nd; ++d)
      if (b.lo[d] < lo[d] || b.hi[d] > hi[d]) return false;
    return true;
  }
};
bool intersects(const Box& a, const Box& b);
Box intersect(const Box& a, const Box& b);
// a minus b as disjoint boxes (slab decomposition, at most 2*nd pieces).
std::vector<Box> subtract(const Box& a, const Box& b);

// ---- grid -------------------------------------------------------------------
struct Block {
  Box full, data;
  int64_t first_cell = 0;
  int64_t stride[HBC_MAX_DIM] = {0};  // cell strides of the full box (row-major)
  int64_t cells = 0;
};

struct Grid {
  int nd = 0;
  int64_t lo[HBC_MAX_DIM] = {0}, hi[HBC_MAX_DIM] = {0};
  // Lattice of stepped slices (Sec. IV-A-1): along dimension d the grid's
  // points are the positions res[d] + step[d] * k, and everything inside the
  // library (lo, hi, blocks, boxes, cells) is in the index k.  Set by the
  // first block added through the C ABI; the global box in positions is
  // [plo, phi).  The identity lattice (step 1, res 0) leaves positions as
  // they are.
  int64_t step[HBC_MAX_DIM] = {1, 1, 1, 1, 1, 1}, res[HBC_MAX_DIM] = {0};
  int64_t plo[HBC_MAX_DIM] = {0}, phi[HBC_MAX_DIM] = {0};
  bool lattice_set = false;
  bool identity_lattice() const {
    for (int d = 0; d < nd; ++d)
      if (step[d] != 1 || res[d] != 0) return false;
    return true;
  }
  std::vector<Block> blocks;
  int64_t ncells = 0;
  int owner(const int64_t* c) const;          // block whose full box holds c, or -1
  int64_t cell(int b, const int64_t* c) const;  // cell number (c inside block b's full box)
  // global linear index over [lo, hi) -> multi-index; false if out of the box
  bool unlinear(int64_t lin, int64_t* c) const;
  int64_t ghost_cells() const;
};

// ---- program ----------------------------------------------------------------
enum SubKind { SUB_MAP = 0, SUB_ZERO = 1, SUB_ELL = 2, SUB_CSR = 3, SUB_VEC = 4, SUB_ZERO_REST = 5 };

struct Sub {
  int kind = SUB_ZERO;
  Box rows;
  int block = -1;  // owner block of the rows (ZERO_REST: the block)
  // map
  int64_t M[HBC_MAX_DIM * HBC_MAX_DIM] = {0};
  int64_t off[HBC_MAX_DIM] = {0};
  double w = 1.0;
  int rot = 0;  // component rotation code
  // ell
  int width = 0;
  std::vector<int64_t> cols;  // global linear (ELL: rows*width; CSR: nnz)
  std::vector<double> vals;
  std::vector<int64_t> ptr;   // CSR
  // vector
  int64_t ninner = 1;
  std::vector<double> b;
};

// A closed component of data rows (block-edge averaging: one co-located set):
// its distinct columns (cells) and its rows [first_row, first_row + nrow) of
// the component row tables.
constexpr int DC_MAX = 8;
struct alignas(16) DataComp {
  int32_t ncol, nrow, first_row, pad_;
  int32_t col[DC_MAX];
};

// Rows on data cells (block-edge averaging): CSR over a box of one block's
// data region, columns as global linear data indices.
struct DataSub {
  Box rows;
  std::vector<int64_t> ptr, cols;
  std::vector<double> vals;
};

struct Program {
  Grid grid;
  std::vector<Sub> subs;
  std::vector<DataSub> dsubs;
  uint32_t flags = 0;
  std::vector<int64_t> consumer;  // consumer read offsets, noffsets x nd (empty: keep every row)
};

// Component rotation codes.  A 2x2 signed permutation R acts on the vector
// slots as out_a = sign_a * in_{p(a)}.  Code bits: 1 = swap (p(0) = 1),
// 2 = sign_0 negative, 4 = sign_1 negative.  Code 0 is the identity.
int rot_code(const int32_t* R);  // -1 if R is not a signed permutation
int rot_inverse(int code);
void rot_matrix(int code, int32_t* R);

// ---- device-facing tables ---------------------------------------------------
enum SegKind { SEG_ZERO = 0, SEG_MAP = 1, SEG_ELL = 2, SEG_CSR = 3, SEG_VEC = 4, SEG_DATA_ROW = 5 };
constexpr int SEG_MAXD = 4;

struct alignas(16) DevSeg {
  int32_t kind;
  int32_t nd;          // box dims after dropping extent-1 dims (1..SEG_MAXD)
  int32_t rot;         // component rotation code
  int32_t has_b;
  int32_t ext[SEG_MAXD];
  int64_t dst_base;    // cell of the box origin
  int64_t dst_stride[SEG_MAXD];
  int64_t src_base;    // MAP: source cell of the box origin
  int64_t src_stride[SEG_MAXD];
  double w;            // MAP weight (stored in FP64; FP32 plans round it)
  int64_t tab;         // ELL/CSR: first table row of this segment
  int64_t brow;        // first row of this segment in the b table
  int32_t width;       // ELL width
  int32_t b_inner;     // 1 or inner
  int64_t nrows;
  int64_t row_base;    // first row of this segment in the plan's row numbering
  int32_t flags;       // SEGF_* bits
  int32_t pad_;
};
constexpr int32_t SEGF_ELL_PADDED = 1;  // some ELL entry is padding (column -1)

struct alignas(16) DevTile {
  int32_t seg;
  int32_t nrows;
  int64_t row0;  // first row within the segment
};

// Point-major work tile: a run of rows of one segment, described by value so
// that the kernel reads it with scalar loads; the rows' cells come from the
// per-row tables (row_dst, row_src) at [row_begin, row_begin + nrows).
struct alignas(16) RowTile {
  int32_t kind;
  int32_t rot;
  int32_t flags;
  int32_t width;      // ELL width
  int64_t row_begin;  // index into the per-row tables
  int64_t tab;        // ELL: element offset of the first row's entries; CSR: index of its row pointer
  int64_t brow;       // b table offset of the first row (has_b)
  double w;           // MAP weight
  int32_t nrows;
  int32_t has_b;
  int32_t b_inner;
  int32_t pad_;
};

// Wide rows (CSR segments averaging >= WIDE_NNZ entries per row, rows of
// >= WIDE_ROW_BYTES, point-major).  A segment's rows are visited with its
// thinnest box dimension innermost (for a halo strip: every ghost layer at one
// tangential position, then the next position), and cut greedily into tiles
// of at most WIDE_ROWS rows whose distinct source cells (at most WIDE_UCAP)
// and entries (at most WIDE_ECAP) fit.  The kernel stages a tile's source
// cells in LDS one slice of inner values at a time (WIDE_ROW_BYTES, or twice
// that for FP64 plans whose layout is 4-aligned); each
// tile has its own copy of its rows' entries (weight, LDS slot of the source)
// and row starts, in tile order.
constexpr int WIDE_NNZ = 8, WIDE_UCAP = 128, WIDE_ROWS = 32, WIDE_ROW_BYTES = 128, WIDE_ECAP = 512;
struct alignas(16) WideTile {
  int32_t rot, has_b, b_inner, nrows;
  int64_t row_base;  // the segment's first row in the per-row tables
  int64_t brow;      // the segment's first row in the b table
  int32_t first_u, nu;  // distinct source cells: w_ucell[first_u, first_u + nu)
  int32_t e0, ne;       // entries: w_ent*[e0, e0 + ne)
  int32_t r0, rp0;      // rows: w_row[r0, r0 + nrows); row starts: w_rp[rp0, rp0 + nrows]
};

// Narrow wide rows: CSR segments averaging >= WIDE_NNZ entries per row whose
// rows are shorter than NARROW_ROW_BYTES (point-major).  A group of
// NARROW_LANES lanes takes one row and splits its entries (lane j takes
// entries j, j + NARROW_LANES, ...), each lane keeps partial sums of every
// inner slot, and the partials are added across the group by a fixed xor
// butterfly.  Tiles are runs of NARROW_ROWS consecutive rows (one workgroup).
constexpr int NARROW_LANES = 16, NARROW_ROW_BYTES = 32, NARROW_ROWS = 256 / NARROW_LANES;
struct alignas(16) NarrowTile {
  int32_t rot, has_b, b_inner, nrows;
  int64_t row_begin;  // index into the per-row tables
  int64_t tab;        // index of the first row's CSR pointer
  int64_t brow;       // b table offset of the first row
};

// Sliding-window rows: 4-wide ELL segments (point-major, whole 16-byte
// vectors, rows of at least WIN_MIN_BYTES) in which every row reads four
// consecutive points of one grid line (the 4-point Lagrange rows of a
// face-edge strip).  Their rows are cut, in device order, into runs of at
// most rows_per_tile (<= WIN_MAXR) rows in which each row's window starts one
// point further along the line than the previous row's: row r of a run reads
// the cells src0 + (r + m) * dl, m < 4, so a run of R rows reads R + 3
// distinct cells.  One wavefront takes a run and a slice of 64 16-byte
// vectors of the inner values and loads each of the run's cells once.
// rows of 256 bytes and up: the window kernel beats the row kernel from there
// (C768 x 32 FP64: 7.4 against 8.6 us); at 128 bytes a wavefront's slice is
// mostly idle lanes and it loses (FP32: 6.7 against 4.8 us)
constexpr int WIN_MAXR = 16, WIN_MIN_BYTES = 256, WIN_DEFAULT_ROWS = 8;
// segments with b: from 512 bytes (C768 x 32 FP64 with b on every strip row:
// 12.4 us windowed at 256 bytes against 10.7 us with the row kernel)
constexpr int WIN_MIN_BYTES_B = 512;
struct alignas(16) WinRun {
  int32_t src0, dl, nrows, nsrc;
  int64_t row_begin;  // first row in the per-row tables (row_dst)
  int64_t tab;        // element offset of the first row's ELL entries
  int64_t brow;       // b table offset of the first row (has_b)
  int32_t rot, has_b, b_inner, pad_;
};

// Adjoint: one entry per (source cell, ghost row) contribution, sorted by
// source cell then ghost cell.
struct CscHost {
  std::vector<int64_t> src_cell;  // distinct source cells, ascending
  std::vector<int64_t> ptr;       // entries of src k: ptr[k] .. ptr[k+1]-1
  std::vector<int64_t> ghost;     // ghost cell of each entry
  std::vector<double> w;          // weight of each entry
  std::vector<int32_t> rot;       // inverse rotation code of each entry
  // Fixed-width copy (width aw = largest entry count, at most ADJ_MAXW): the
  // entries of source k at k*aw + m, m < cnt[k], so that a source's entries
  // are addressed without reading ptr first.  Sources with cnt > aw use the
  // CSR form above.
  int32_t aw = 0;
  std::vector<int32_t> cnt;
  std::vector<int32_t> fghost;
  std::vector<double> fw;
  std::vector<int8_t> frot;
};
constexpr int ADJ_MAXW = 8;
// Row groups of at least this many lanes (rows of >= 128 bytes) take
// contiguous runs of rows (neighbouring rows share sources); narrower groups
// take rows round-robin (neighbouring lanes write neighbouring cells).
constexpr int CHUNK_LPR = 8;
// Rows a row group handles per batch (all their loads issued together).
inline int rows_per_batch(int lanes_per_row) { return lanes_per_row >= 128 ? 2 : 4; }

// LDS-staged adjoint (point-major plans).  A tile is a run of consecutive
// sources; the distinct ghost rows its entries read (at most ADJ_LDS_ROWS,
// and at most the LDS budget) are loaded once into LDS, and each entry holds
// the LDS slot of its ghost.  A ghost row read by one tile only is zeroed by
// that tile once loaded; one read by several tiles has a counter of reader
// tiles, and the tile whose decrement empties it zeroes the row and restores
// the counter for the next call.  Covered ghost rows no source reads are
// zeroed by extra workgroups of the same launch.
constexpr int ADJ_LDS_ROWS = 64;  // 32..160 measured: 64 is fastest at C768 x 32
constexpr int ADJ_LDS_BLOCK = 256;  // threads of the LDS adjoint's workgroups
constexpr int ADJ_LDS_BYTES = 40 * 1024;
constexpr int ADJ_ZERO_ROWS = 64;  // rows per zeroing workgroup
// Reader counters the allocation-free adjoint keeps in its static device
// array (4 MiB).
constexpr int ADJ_NOALLOC_COUNTERS = 1 << 20;
struct AdjLdsTile {
  int32_t first_src, nsrc, first_u, nu;
};
struct AdjLdsHost {
  bool ok = false;
  int32_t brows = 0;                // LDS rows per tile
  std::vector<AdjLdsTile> tiles;
  std::vector<int32_t> u_cell;      // distinct ghost rows of each tile
  std::vector<int32_t> u_ctr;       // counter of a row several tiles read, else -1
  std::vector<int32_t> ctr_init;    // reader tiles per counter
  std::vector<uint16_t> slot;       // per source k, entry m < cnt[k]: LDS slot, at k*aw + m
  std::vector<int32_t> zero_rows;   // covered ghost rows that no source reads
};

struct AdjTile {
  int32_t first;  // first source index
  int32_t count;
};

struct HostTables {
  std::vector<DevSeg> segs;
  std::vector<DevTile> tiles;
  std::vector<int32_t> ell_col;  // cell numbers, -1 padding
  std::vector<double> ell_val;
  std::vector<int64_t> csr_ptr;  // per CSR table row, absolute into csr_col
  std::vector<int32_t> csr_col;
  std::vector<double> csr_val;
  std::vector<double> bval;      // b table: rows * b_inner (per segment)
  std::vector<Box> seg_box;      // each segment's rows in global coordinates
  std::vector<std::vector<int>> seg_order;  // global dims of the segment rows, slowest first
  CscHost csc;
  std::vector<AdjTile> adj_tiles;
  AdjLdsHost adj_lds;
  // point-major row tables (device order) and tiles
  std::vector<int32_t> row_dst;  // destination cell of every covered row
  std::vector<int32_t> row_src;  // MAP rows: source cell; other rows: 0
  std::vector<RowTile> rtiles;
  // wide rows (see WideTile); seg_wide marks the segments they take
  std::vector<char> seg_wide;
  std::vector<WideTile> wtiles;
  std::vector<int32_t> w_ucell;
  std::vector<int32_t> w_row;    // segment-relative row of each tile row
  std::vector<int32_t> w_rp;     // per tile: nrows + 1 row starts, relative to the tile's e0
  std::vector<double> w_entw;    // entries in tile order: weight
  std::vector<int32_t> w_ents;   // entries in tile order: LDS slot of the source cell
  int32_t w_maxu = 0, w_maxe = 0;  // largest nu and ne over the tiles (LDS sizing)
  // narrow wide rows (see NarrowTile); seg_narrow marks the segments they take
  std::vector<char> seg_narrow;
  std::vector<NarrowTile> ntiles;
  // sliding-window rows (see WinRun); seg_win marks the segments they take
  std::vector<char> seg_win;
  std::vector<WinRun> wruns;
  int32_t win_maxr = 0;  // longest run
  bool win_has_b = false;  // a run with b values (the window launch picks its instance by it)
  // data rows: destination cells, CSR over data cells (absolute pointers)
  std::vector<int32_t> dr_cell;
  std::vector<int64_t> dr_ptr;
  std::vector<int32_t> dr_col;
  std::vector<double> dr_val;
  // the data rows split into closed components (rows that read each other's
  // cells), each small enough to be read into registers whole, then written
  bool dc_ok = false;
  std::vector<DataComp> dc_comp;
  std::vector<int32_t> dc_row_dst, dc_row_ent, dc_row_n;  // per component row
  std::vector<int32_t> dc_slot;                           // per entry: column slot in its component
  std::vector<double> dc_w;
};

struct Layout {
  int64_t inner = 1;
  int order = HBC_POINT_MAJOR;
  int64_t vec_len = 0, vec_lo = 0, vec_stride = 0;
};

// The b values of one segment as plan compile laid them out: the rows of
// `box` visited in `order`, bi values per row at host.bval[brow + q * bi + l],
// each the sum, in the order of `vecs`, of those sub-vectors' values
// (indices into Plan::vsubs).
struct BSeg {
  Box box;
  std::vector<int> order;
  std::vector<int> vecs;
  int64_t bi = 1;
  int64_t brow = 0;
};

struct Plan {
  Grid grid;
  Layout layout;
  int dtype = HBC_F64;
  uint32_t flags = 0;
  HostTables host;
  std::vector<Sub> vsubs;        // the program's sub-vectors, values as last set
  std::vector<int32_t> vsub_id;  // their ids in the program
  std::vector<BSeg> bsegs;       // segments with b
  hbc_stats stats{};
  hbc_tune tune{};
  int vec = 1;     // elements per lane access (point-major)
  int unroll = 1;  // accesses per lane and row: vec * unroll elements make 16 bytes where the row allows
  // device storage: one allocation holding every table
  void* dev = nullptr;
  size_t dev_bytes = 0;
  const DevSeg* d_segs = nullptr;
  const DevTile* d_tiles = nullptr;
  const RowTile* d_rtiles = nullptr;
  const int32_t* d_row_dst = nullptr;
  const int32_t* d_row_src = nullptr;
  const int32_t* d_ell_col = nullptr;
  const void* d_ell_val = nullptr;
  const int64_t* d_csr_ptr = nullptr;
  const int32_t* d_csr_col = nullptr;
  const void* d_csr_val = nullptr;
  const void* d_bval = nullptr;
  const WideTile* d_wtiles = nullptr;
  const int32_t* d_w_ucell = nullptr;
  const int32_t* d_w_row = nullptr;
  const int32_t* d_w_rp = nullptr;
  const void* d_w_ent = nullptr;  // packed {weight, slot * values per slice} per entry
  const NarrowTile* d_ntiles = nullptr;
  const WinRun* d_wruns = nullptr;  // in the tile allocation (depends on the launch shape)
  uint64_t tile_gen = 0;            // bumped whenever the tile tables are rebuilt on the device
  const int32_t* d_dr_cell = nullptr;
  const int64_t* d_dr_ptr = nullptr;
  const int32_t* d_dr_col = nullptr;
  const void* d_dr_val = nullptr;
  void* d_dr_scratch = nullptr;  // rows_data * inner values (own allocation)
  const DataComp* d_dc_comp = nullptr;
  const int32_t* d_dc_row_dst = nullptr;
  const int32_t* d_dc_row_ent = nullptr;
  const int32_t* d_dc_row_n = nullptr;
  const int32_t* d_dc_slot = nullptr;
  const void* d_dc_w = nullptr;
  void* d_csc_dev = nullptr;  // allocation holding the adjoint tables
  const int64_t* d_csc_src = nullptr;
  const int64_t* d_csc_ptr = nullptr;
  const int64_t* d_csc_ghost = nullptr;
  const void* d_csc_w = nullptr;
  const int32_t* d_csc_rot = nullptr;
  const int32_t* d_adj_cnt = nullptr;
  const int32_t* d_adj_fg = nullptr;
  const void* d_adj_fw = nullptr;
  const int8_t* d_adj_frot = nullptr;
  void* d_al_dev = nullptr;  // allocation holding the LDS-staged adjoint tables
  const AdjLdsTile* d_al_tiles = nullptr;
  const int32_t* d_al_ucell = nullptr;
  const int32_t* d_al_uctr = nullptr;
  const int32_t* d_al_ctrinit = nullptr;
  int32_t* d_al_ctr = nullptr;  // reader counters (restored by every adjoint call)
  const uint16_t* d_al_slot = nullptr;
  const int32_t* d_al_zero = nullptr;
  const AdjTile* d_adj_tiles = nullptr;
  // 27-point consumer: per block and neighbour direction, the block the BC
  // copies from (-1 zero rows, -2 uncovered); computed at plan creation.
  // st_ok: the grid suits the stencil (equal blocks, one-cell halo, inner 1);
  // st_fused: the BC can also be read through st_info by the fused form.
  bool st_ok = false, st_fused = false;
  std::string st_reason, st_fused_reason;
  std::vector<int64_t> st_info;
  const int64_t* d_st_info = nullptr;
  void* d_st_dev = nullptr;
  int64_t st_n[3] = {0, 0, 0};
  int st_nblocks = 0;
};

// ---- consumer: the operator that reads the BC's ghosts (Sec. IV-C) ----------
// y[c, l] = sum_o w_o x'[c + o, l] for every data cell c of every block, with
// x' the field after the apply.  Structured tiles cover runs of cells along the
// last dimension of a block's data box and read x at c + o directly (every
// read a data cell, or a ghost already stored); the boundary rows of the fused
// form are the stencil composed with the BC rows of the ghosts it reaches:
// entries (source cell, w_o * A[g, k], the ghost row's component rotation) in
// offset order then BC entry order, plus sum_o w_o b[g] per row.
struct alignas(16) CTile {
  int32_t cell0;  // first cell of the run
  int32_t y0;     // its row in the output (data cells block by block, each data box row-major)
  int32_t n;      // cells
  int32_t blk;    // block (cell deltas of the offsets)
};
constexpr int CONS_RB = 2;      // cells per batch of a row group (the batch walk)
// boundary rows per row group and tile: 8 keeps the composed rows' tiles few
// (C384 x 256 cross: 575 workgroups before the structured tiles, 762 us fused
// against 780 us with one row per group, which made 4596 workgroups of
// latency-bound gathers)
constexpr int CONS_BROWS = 8;
constexpr int CONS_CELLS = 16;  // cells of a structured tile per row group
constexpr int CONS_MAXOFF = 64; // offsets at most
constexpr int CONS_MAXLINES = 3; // lines of the line walk at most
struct ConsumerHost {
  int noff = 0;
  std::vector<int64_t> off;        // noff x nd, lattice steps (line by line when nlines > 0)
  std::vector<double> w;           // noff
  std::vector<int32_t> delta;      // nblocks x noff cell deltas
  // line walk of the structured tiles: the offsets lie on nlines lines along
  // the last dimension (equal in the others), each within +-1 along it; a
  // row group keeps the last three points of each line in registers.  0: the
  // general walk.
  int nlines = 0;
  std::vector<int32_t> line_delta; // nblocks x nlines: cell delta of each line's last point
  std::vector<double> line_w;      // nlines x 3: weight of ring slot s (the line's last point - 2 + s)
  int32_t line_mask = 0;           // bit 3 l + s: slot s of line l is an offset
  std::vector<CTile> tiles_all;    // every data cell (unfused: ghosts read from the field)
  std::vector<CTile> tiles_int;    // cells whose reads are all data cells (fused)
  std::vector<int32_t> brow_y;     // boundary rows (fused): output row
  std::vector<int32_t> bptr;       // entries [bptr[r], bptr[r + 1])
  std::vector<int32_t> bcol;
  std::vector<double> bw;
  std::vector<int8_t> brot;
  std::vector<int32_t> bconst_row; // per boundary row: row of bconst, or -1
  std::vector<double> bconst;      // rows x inner
  int32_t tile_cells = 0;          // cells per structured tile (row groups x CONS_CELLS)
  int32_t tile_rows = 0;           // boundary rows per tile (row groups x CONS_BROWS)
  int64_t ndata = 0;
};

// host plan compiler (plan.cpp)
void compile_plan(const Program& prog, const Layout& lay, int dtype, Plan& plan);
void build_tiles(Plan& plan, const hbc_tune& t);
hbc_tune default_tune(const Plan& plan);
bool windows_possible(const Plan& plan);
void build_csc(Plan& plan);
void compute_stencil_info(Plan& plan);
// new values for sub-vector sub_id: recomputes the b values it contributes
// to; returns the changed range [first, last) of host.bval (empty if none)
std::pair<int64_t, int64_t> plan_set_vector(Plan& plan, int32_t sub_id, const double* values);
// host evaluation of a compiled row
int plan_row(const Plan& plan, int64_t cell, int64_t l, int cap, int64_t* cols, double* vals, int32_t* nnz,
             double* b, int32_t* kind, int32_t* rot);

// consumer compile (consumer.cpp): offsets in positions of the global box
void compile_consumer(const Plan& plan, int noff, const int64_t* offsets, const double* weights, ConsumerHost& C);

// cubed sphere helpers (cubed_sphere.cpp)
void cs_add_program(Program& p, int64_t N, int64_t h, int mode, int vector, const int32_t* base,
                    const double* w);
// Cartesian helpers (cubed_sphere.cpp)
void cart_add_halo(Program& p, const int32_t* nb, const int64_t* n, int64_t h, int32_t periodic);
void cs_add_edge_average(Program& p, int64_t Np);
void cs_add_quadrature(Program& p, int64_t N, int64_t h, int q, int vector);

}  // namespace hbc
