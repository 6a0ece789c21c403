/*
 * hbc.h — C ABI of hipbc: boundary conditions as affine sparse operators,
 * ghost = A * interior + b, on block-structured grids, for MI355X (gfx950).
 *
 * Model (Mat2Boundary, arXiv 2605.14780):
 *  - Sec. III-A: every variable lives on a full region = data region + ghost
 *    region.  Sec. IV-A-1: one global box [lo, hi) per dimension; each block's
 *    full and data regions are slices (start, stop, step) of it, ghost = full -
 *    data.  Alg. 1 puts the block id in the leading coordinate, so block full
 *    regions are disjoint in global coordinates (checked here).
 *  - Sec. III-B: a BC is F(x) = A x + b with x over the data region; the six
 *    BC kinds of that section become rows of A / entries of b.
 *  - Sec. IV-A-3 (Table II) and IV-A-4 (Table III): A is split into basic
 *    sub-matrices, each valid on a set of rows and giving a row iterator:
 *    a static list (here: one affine map entry, or none) or a dynamic
 *    iterator (here: ELL or CSR tables).  A basic sub-vector gives b.
 *
 * Storage of a field (the device array the apply works on): cells are
 * numbered block by block in creation order, each block's full box in
 * row-major order (last coordinate fastest); hbc_grid_block_cells() gives each
 * block's first cell number.  Every cell holds `inner` values (levels x fields
 * x components).  POINT_MAJOR stores value (cell, l) at cell*inner + l;
 * PLANE_MAJOR at l*ncells + cell.
 *
 * Conventions for every call:
 *  - Return 0 (HBC_OK) or a negative HBC_E* code; hbc_last_error() then holds
 *    a message (thread-local).  No call aborts and no C++ exception escapes.
 *  - Host arrays passed in are copied before the call returns; the caller may
 *    free them immediately.
 *  - Device pointers (fields, outputs) are borrowed: the caller keeps them
 *    alive until the stream has passed the call.  Field base pointers must be
 *    16-byte aligned.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  Apply
 *    calls are asynchronous on that stream.
 *  - Plans are immutable after creation (apart from tuning and new sub-vector
 *    values, hbc_plan_set_vector), so applies on different streams may run
 *    concurrently on different fields.  The exceptions are the adjoint (calls
 *    of hbc_apply_adjoint on one plan must not overlap in time, see there)
 *    and hbc_plan_set_vector, which no work on another stream that uses the
 *    plan may overlap.
 *  - destroy(NULL) is a no-op.
 */
#ifndef HBC_H
#define HBC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HBC_MAX_DIM 6

/* status codes */
#define HBC_OK 0
#define HBC_EINVAL (-1)      /* bad argument, slice, size or null pointer */
#define HBC_ERANGE (-2)      /* row outside its block's ghost region, or column outside every data region */
#define HBC_EOVERLAP (-3)    /* overlapping sub-matrix (or sub-vector) rows without HBC_ALLOW_OVERLAP_SUM */
#define HBC_EALIAS (-4)      /* a row written is also read as a column (in-place hazard) */
#define HBC_EUNCOVERED (-5)  /* ghost rows covered by nothing under HBC_STRICT_COVER */
#define HBC_ENOMEM (-6)      /* host or device allocation failed */
#define HBC_EHIP (-7)        /* a HIP runtime error; its string is in hbc_last_error() */
#define HBC_EUNSUPPORTED (-8)/* valid request outside what the library implements (e.g. a block whose step differs from the grid's lattice) */

/* element types */
#define HBC_F64 0
#define HBC_F32 1

/* field layouts */
#define HBC_POINT_MAJOR 0
#define HBC_PLANE_MAJOR 1

/* program flags */
#define HBC_STRICT_COVER 1u        /* every ghost cell must be covered by a sub-matrix or sub-vector */
#define HBC_ALLOW_OVERLAP_SUM 2u   /* overlapping rows add their contributions (default: HBC_EOVERLAP) */

/* plan flags */
#define HBC_PLAN_HOST_ONLY 1u      /* compile and validate only; no device tables (no GPU needed) */
#define HBC_PLAN_NO_WINDOWS 2u     /* serve sliding-window rows (see hbc_stats.rows_window) with the general
                                      row kernel instead of the window kernel; results are bit-identical */

/* cubed-sphere program modes */
#define HBC_CS_SYNC 0              /* rotated halo copy of the neighbour's cell */
#define HBC_CS_LAGRANGE 1          /* 4-point Lagrange along the neighbour's grid line */

typedef struct hbc_grid hbc_grid;
typedef struct hbc_program hbc_program;
typedef struct hbc_plan hbc_plan;
typedef struct hbc_batch hbc_batch;

/* One slice (start, stop, step) of a dimension, Sec. IV-A-1. */
typedef struct {
  int64_t start, stop, step;
} hbc_slice;

/* Half-open box of row multi-indices; the first `ndim` entries are used. */
typedef struct {
  int64_t lo[HBC_MAX_DIM];
  int64_t hi[HBC_MAX_DIM];
} hbc_box;

/* Storage layout of the fields a plan is applied to.
 * inner:      values per cell (>= 1).
 * order:      HBC_POINT_MAJOR or HBC_PLANE_MAJOR.
 * vec_len:    0, or the number of slots of each component of one 2-component
 *             vector field: component 0 = slots [vec_lo, vec_lo + vec_len),
 *             component 1 = slots [vec_lo + vec_stride, ... + vec_len).
 *             Sub-matrices with a component rotation act on these slots
 *             (Sec. V-A: multi-component vectors per grid point). */
typedef struct {
  int64_t inner;
  int32_t order;
  int32_t vec_len;
  int64_t vec_lo;
  int64_t vec_stride;
} hbc_layout;

/* Plan statistics (per apply, per field). */
typedef struct {
  int64_t ghost_cells;      /* all ghost cells of the grid */
  int64_t rows_covered;     /* ghost rows written by an apply */
  int64_t rows_uncovered;   /* ghost rows left unchanged */
  int64_t rows_zero, rows_map, rows_ell, rows_csr, rows_vector_only;
  int64_t rows_with_b;
  int64_t nnz;              /* stored entries of A (ELL padding excluded) */
  int64_t unique_sources;   /* distinct data cells read by A */
  int64_t segments, tiles;
  int64_t ghost_values;     /* rows_covered * inner */
  double alg_bytes;         /* ghost writes + unique source reads + b + tables, per apply */
  double alg_bytes_adjoint; /* ghost reads + ghost zeroing + source read-modify-write + tables */
  int64_t table_bytes;      /* device bytes held by the plan */
  int64_t rows_data;        /* data rows written (block-edge averaging), staged through scratch */
  int64_t rows_dead;        /* ghost rows of sub-matrices / sub-vectors dropped: no consumer read reaches them */
  int64_t ghost_cells_live; /* ghost cells some consumer read reaches (all ghost cells without a consumer) */
  int64_t rows_wide;        /* CSR rows served by the LDS-staged wide-row kernel (point-major, >= 128-byte rows) */
  int64_t wide_tiles;       /* tiles of those rows */
  int64_t rows_narrow;      /* CSR rows of >= 8 entries and < 32 bytes served by the entry-splitting kernel */
  int64_t rows_window;      /* 4-entry rows on four consecutive points of a grid line, each row's window at
                               the previous row's or one point further (Sec. III-B interpolation rows of a
                               face-edge strip), served by the window kernel: point-major, rows of >= 256
                               bytes in whole 16-byte vectors; each wavefront loads a run's cells once */
  int64_t window_runs;      /* runs of those rows (at most rows_per_tile rows each) */
} hbc_stats;

/* Launch shape of the apply kernels (chosen by the plan, changed by tuning).
 * The point-major adjoint's LDS kernel has a fixed shape of its own (256
 * threads, about 4 lanes per row); the other adjoint kernels follow this one. */
typedef struct {
  int32_t block;            /* threads per workgroup: 64, 128, 192 or 256 */
  int32_t lanes_per_row;    /* power of two; lanes that share one row */
  int32_t rows_per_tile;    /* rows per work tile (sliding-window rows: rows per run, at most 16) */
  int32_t persistent;       /* 0: one workgroup per tile; >0: that many workgroups loop over tiles */
  int32_t window_order;     /* sliding-window rows: 0 pipelined (each row's store issued while later
                               rows' sources still arrive), 1 ordered (sources, then the rows in turn);
                               both give the same bits */
} hbc_tune;

/* ---- errors ---------------------------------------------------------------- */
/* Message of the last failing call on this thread ("" if none).  Owned by the library. */
const char* hbc_last_error(void);

/* ---- grid and block layout (Sec. III-A, IV-A-1, Alg. 1) ---------------------- */
/* Create a grid over the global box [lo[d], hi[d]), d < ndim (1 <= ndim <= 6). */
int hbc_grid_create(int32_t ndim, const int64_t* lo, const int64_t* hi, hbc_grid** out);
/* Add a block: full and data are ndim slices; data inside full, full inside the
 * global box, full regions of different blocks disjoint.  A slice (start, stop,
 * step) selects the points start + k*step < stop (Sec. IV-A-1: step 2 for a
 * staggered variable, 2^k for a multigrid level); the block's cells are the
 * points of its full slices, its data cells those of its data slices.  The
 * first block fixes the grid's lattice: along each dimension every full and
 * data slice of the grid must have that block's step and a start congruent to
 * its start modulo the step (HBC_EUNSUPPORTED otherwise).  Every position later
 * given to a program on this grid (row boxes, map matrices and offsets,
 * columns, consumer offsets) is a position of the global box: a row box
 * selects the grid points it holds, columns must be grid points (HBC_ERANGE),
 * a map must send grid points to grid points and consumer offsets must be
 * multiples of the step (HBC_EINVAL).  *block_id receives the block's index. */
int hbc_grid_add_block(hbc_grid* g, const hbc_slice* full, const hbc_slice* data, int32_t* block_id);
/* Total cells of all blocks' full regions (the field's cell count). */
int64_t hbc_grid_cells(const hbc_grid* g);
/* First cell number and cell count of block b's full region. */
int hbc_grid_block_cells(const hbc_grid* g, int32_t b, int64_t* first_cell, int64_t* ncells);
void hbc_grid_destroy(hbc_grid* g);

/* Cubed sphere (equiangular gnomonic): 6 blocks along coordinate 0, block f has
 * full (f, f+1) x [-h, N+h)^2 and data (f, f+1) x [0, N)^2; index (face, j, i).
 * N >= 4 and 1 <= h <= N/2: a ghost layer's centre angle pi/4 + (k + 1/2) pi/(2N)
 * must stay below pi/2, inside the face's gnomonic chart (HBC_EINVAL otherwise;
 * the same bound holds for every cubed-sphere entry point). */
int hbc_cs_grid_create(int64_t N, int64_t h, hbc_grid** out);
/* Cartesian multi-block: nb[0]*nb[1]*nb[2] blocks of n[0] x n[1] x n[2] data cells
 * with halo h, block id b = (bz*nb1 + by)*nb2 + bx along coordinate 0, then (z, y, x). */
int hbc_cart_grid_create(const int32_t* nb, const int64_t* n, int64_t h, hbc_grid** out);

/* ---- BC program: basic sub-matrices / sub-vectors (Sec. IV-A-3, Tables II, III) */
/* The program keeps its own copy of the grid. */
int hbc_program_create(const hbc_grid* g, hbc_program** out);
void hbc_program_destroy(hbc_program* p);
int hbc_program_set_flags(hbc_program* p, uint32_t flags);

/* Static one-entry rows: for each row multi-index r in `rows`,
 *   A[r, M r + offset] = weight,
 * M an ndim x ndim integer matrix (row-major), offset ndim integers.  Covers
 * halo copy, circular / symmetric maps and rotated copies (Sec. III-B; Alg. 1's
 * right ghost).  `rot` is NULL or a 2x2 signed permutation (row-major) applied
 * to the vector components of the layout.  The image of the box must lie in
 * one block's data region (HBC_ERANGE). */
int hbc_program_add_map(hbc_program* p, const hbc_box* rows, const int64_t* M, const int64_t* offset,
                        double weight, const int32_t* rot, int32_t* sub_id);
/* Number of rows (grid points) the row box `rows` selects: the row count k
 * runs over in add_ell, add_csr, add_vector and add_data_csr (on a grid of
 * stepped slices, the lattice points inside the box). */
int hbc_program_box_rows(const hbc_program* p, const hbc_box* rows, int64_t* n);
/* Rows with no entries: padding with zeros (Sec. III-B); written as +0.0. */
int hbc_program_add_zero(hbc_program* p, const hbc_box* rows, int32_t* sub_id);
/* Zero rows for every ghost cell of `block` that no other sub-matrix covers,
 * resolved when the plan is compiled (the complement region of Alg. 1). */
int hbc_program_add_zero_rest(hbc_program* p, int32_t block, int32_t* sub_id);
/* Fixed-width rows (ELL): row k of the box (row-major) has entries
 * (cols[k*width + m], vals[k*width + m]), m < width; cols are row-major linear
 * indices over the global box of data cells, -1 marks padding. */
int hbc_program_add_ell(hbc_program* p, const hbc_box* rows, int32_t width, const int64_t* cols,
                        const double* vals, const int32_t* rot, int32_t* sub_id);
/* Variable-width rows (CSR, Alg. 1's BoundaryCSR): row k has entries
 * row_ptr[k] .. row_ptr[k+1]-1 of cols / vals (global linear data indices). */
int hbc_program_add_csr(hbc_program* p, const hbc_box* rows, const int64_t* row_ptr, const int64_t* cols,
                        const double* vals, const int32_t* rot, int32_t* sub_id);
/* Basic sub-vector: b over `rows`, values[k*ninner + l] for row k (row-major);
 * ninner is 1 (same b for every inner slot) or the layout's inner extent. */
int hbc_program_add_vector(hbc_program* p, const hbc_box* rows, int64_t ninner, const double* values,
                           int32_t* sub_id);

/* Consumer footprint (Sec. IV-C: boundary writes that no later read depends
 * on are removed, and the rest is split into disjoint boxes).  `offsets`
 * (noffsets x ndim, row-major) are the relative positions at which the
 * operator consuming the field reads around each data cell.  A ghost cell is
 * live if a data cell of its block plus some offset lands on it; rows of
 * sub-matrices and sub-vectors at other ghost cells are dropped (not written,
 * counted in rows_dead), and HBC_STRICT_COVER then asks only for the live
 * ghosts to be covered.  noffsets = 0 restores the default (every row kept).
 * Block grids keep offset 0 in the block coordinate. */
int hbc_program_set_consumer(hbc_program* p, int32_t noffsets, const int64_t* offsets);

/* Rows on data cells (Sec. III-B block-edge averaging: where points of
 * different blocks share one physical location, a sparse Sync sub-matrix with
 * a few entries per row rewrites those data values).  `rows` lies in one
 * block's data region; row k has entries row_ptr[k] .. row_ptr[k+1]-1 of
 * cols (global linear data indices) / vals.  Every row of an apply, ghost or
 * data, reads the input values: data rows that read each other's cells form
 * closed components, each read whole into registers and written after the
 * ghost rows (components of up to 8 rows, columns and entries per row);
 * otherwise the data rows are staged through a plan-owned scratch buffer, and
 * applies of such a plan must not overlap in time.  Point-major
 * layouts only; such plans have no adjoint, batch or 27-point consumer
 * (HBC_EUNSUPPORTED).  Data-row boxes may not overlap each other (HBC_EOVERLAP). */
int hbc_program_add_data_csr(hbc_program* p, const hbc_box* rows, const int64_t* row_ptr, const int64_t* cols,
                             const double* vals, int32_t* sub_id);
/* Block-edge averaging on a vertex-centred cubed sphere (grid from
 * hbc_cs_grid_create(Np, h): Np points per face side, the boundary points of a
 * face coincide with its neighbours'): every face-boundary point becomes the
 * mean of its 2 (cube edge) or 3 (cube corner) co-located copies, entries in
 * ascending cell order with weight 1/k.  Connectivity from the integer face
 * frames. */
int hbc_cs_program_add_edge_average(hbc_program* p, int64_t Np);

/* Cubed-sphere programs on a grid from hbc_cs_grid_create (Sec. II-B; Sec. III-B
 * halo copy and user-defined interpolation; Alg. 1's rotated map).  For each of
 * the 24 face sides one sub-matrix over that side's h x N ghost strip, plus 24
 * zero corners.  HBC_CS_SYNC: rotated copy of the neighbour's cell on the
 * mirrored grid line.  HBC_CS_LAGRANGE: 4 entries on that line at
 * base .. base+3 with the given weights, where base[k*N + t] and
 * w[(k*N + t)*4 + m] describe ghost layer k, tangential index t (from
 * hbc_cs_lagrange_weights, copied to the host); NULL for SYNC.  With
 * `vector` != 0 each side carries its 2x2 component rotation. */
int hbc_cs_program_add(hbc_program* p, int64_t N, int64_t h, int32_t mode, int32_t vector,
                       const int32_t* base, const double* w);
/* Wide interpolation rows on a grid from hbc_cs_grid_create (Sec. III-B:
 * HOPE's ghost values as Itp = Agg . Recons, user-preprocessed into sparse
 * rows): each edge ghost cell is the q x q Gauss-Legendre average (q = 1, 2,
 * 3) over its square in its face's angles of cubic tensor-product Lagrange
 * reconstructions (4 x 4 nodes in the neighbour's index space, base
 * clamp(floor(s) - 1, 0, N - 4) per direction); the row is the union of the
 * stencils with weights summed (16..25 entries for q = 2), in ascending cell
 * order, stored as CSR.  Corners are zero rows; `vector` adds the side's
 * component rotation.  Weights from FP64 geometry on the host. */
int hbc_cs_program_add_quadrature(hbc_program* p, int64_t N, int64_t h, int32_t q, int32_t vector);
/* Cartesian halo program on a grid from hbc_cart_grid_create: for every block
 * and each of its 3^3-1 ghost regions, a copy from the neighbouring block
 * (Sec. III-B halo copying) or, outside the domain, zero rows (padding with
 * zeros); bit d of periodic_mask wraps dimension d (z=0, y=1, x=2) instead. */
int hbc_cart_program_add_halo(hbc_program* p, const int32_t* nb, const int64_t* n, int64_t h,
                              int32_t periodic_mask);

/* ---- plan: program compiled for a layout and element type ------------------- */
/* Validates, partitions the rows into disjoint boxes (Sec. IV-B's
 * non-overlapping set; Sec. IV-C's disjoint convex pieces), and builds the
 * device tables.  dtype: HBC_F64 or HBC_F32 (weights rounded to nearest).
 * flags: HBC_PLAN_HOST_ONLY. */
int hbc_plan_create(const hbc_program* p, const hbc_layout* layout, int32_t dtype, uint32_t flags,
                    hbc_plan** out);
void hbc_plan_destroy(hbc_plan* plan);
int hbc_plan_stats(const hbc_plan* plan, hbc_stats* out);
/* Host evaluation of the compiled row of one ghost cell (no GPU): up to `cap`
 * entries (column cell number, weight) and b for inner slot l (0 if none).
 * *nnz receives the row's entry count, *kind its segment kind (0 zero, 1 map,
 * 2 ELL, 3 CSR, 4 b only, 5 data row (hbc_program_add_data_csr; ghost_cell
 * may then name a data cell), -1 uncovered). */
int hbc_plan_row(const hbc_plan* plan, int64_t ghost_cell, int64_t l, int32_t cap, int64_t* cols,
                 double* vals, int32_t* nnz, double* b, int32_t* kind, int32_t* rot);
/* New values for a basic sub-vector of the plan's program (Sec. III-B: the
 * affine part b of F, e.g. a Dirichlet value that changes from step to step),
 * without compiling the plan again.  sub_id is the id hbc_program_add_vector
 * returned; values (host, caller-owned, FP64) has the layout and length given
 * there (rows of the sub-vector's box, row-major, times its ninner).  Every b
 * value the sub-vector contributes to is recomputed as at plan creation (the
 * sum over the sub-vectors covering the row, rounded to the plan's type) and
 * copied to the device, ordered after earlier work on `stream`; the call
 * returns when the copy is done.  Captured graphs and batches holding the
 * plan read the new values from their next launch.  Work on other streams
 * that uses the plan must not overlap the call.  Host-only plans update their
 * host tables (hbc_plan_row).  HBC_EINVAL: sub_id is not a sub-vector of the
 * program, or NULL values for a non-empty sub-vector. */
int hbc_plan_set_vector(hbc_plan* plan, int32_t sub_id, const double* values, void* stream);
int hbc_plan_get_tune(const hbc_plan* plan, hbc_tune* out);
/* Replace the launch shape (rebuilds the tile table).  Results are identical
 * for every valid shape.  Graphs captured from the plan before the call
 * (hbc_graph_create) point at the old tile table: hbc_graph_launch refuses
 * them afterwards (HBC_EINVAL) and they must be captured again; the same
 * holds after hbc_plan_autotune. */
int hbc_plan_set_tune(hbc_plan* plan, const hbc_tune* t);

/* Try candidate launch shapes (workgroup size, lanes per row, rows per tile,
 * persistent workgroups; for plans with sliding-window rows the run length and
 * the order of loads and stores), timing HIP-graph applies cycled over the `nfields`
 * device fields (`nelem` values each; their ghost values are overwritten,
 * data cells are not), and keep the fastest.  With cache_path (JSON lines
 * keyed by device, dtype, layout, the plan's sizes and the generation of the
 * library's kernels) a stored choice is reused; one stored by a build whose
 * kernels time differently is not.  *ms receives the chosen shape's time
 * per apply.  Results do not depend on the shape (Sec. V-C: specialise once,
 * run many). */
int hbc_plan_autotune(hbc_plan* plan, void* const* fields, int64_t nelem, int32_t nfields, const char* cache_path,
                      void* stream, double* ms);

/* ---- apply (Sec. III-B: y = A x + b on the ghost rows) ------------------------ */
/* In place on `field` (device, `nelem` values = cells * inner, else
 * HBC_EINVAL): every covered ghost value := (A x + b); data cells and
 * uncovered ghosts are not written. */
int hbc_apply(const hbc_plan* plan, void* field, int64_t nelem, void* stream);
/* Adjoint, in place on `grad` (device, a full field of output gradients):
 * data cells += A^T * (covered ghost gradients), then covered ghost gradients
 * := 0 (the vector-Jacobian product of hbc_apply; Sec. III-B's F is affine, so
 * its Jacobian is A).  Deterministic: every data value is summed by one thread
 * in ascending ghost order.  One launch: a ghost row that several workgroups
 * read is zeroed by the last of them, found with a per-row counter of reader
 * workgroups that the plan owns and every call restores; adjoint calls on one
 * plan must therefore not overlap in time (serialise them on one stream).
 * The first call builds the transposed tables (allocates; not inside graph
 * capture: hbc_graph_create with HBC_OP_ADJOINT builds them first). */
int hbc_apply_adjoint(const hbc_plan* plan, void* grad, int64_t nelem, void* stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the adjoint
 * of hbc_apply_adjoint, with the same result bit for bit, that allocates
 * nothing.  Its reader counters live in one static device array of 2^20
 * int32 (4 MiB) per GPU, held until the process ends; every call starts them
 * at their reader counts with a small copy kernel on `stream`, so calls on
 * one GPU must not overlap in time (whatever their plans), and they race with
 * each other if they do.  Needs the plan's transposed tables, which the first
 * hbc_apply_adjoint or hbc_graph_create(HBC_OP_ADJOINT) builds (HBC_EINVAL
 * otherwise), and at most 2^20 counters (HBC_EINVAL beyond; hbc_apply_adjoint
 * has no such limit). */
int hbc_apply_adjoint_noalloc(const hbc_plan* plan, void* grad, int64_t nelem, void* stream);
/* The kernels one call of `op` (HBC_OP_APPLY: hbc_apply; HBC_OP_ADJOINT:
 * hbc_apply_adjoint) launches with the plan's current launch shape, in launch
 * order: their demangled names (as profilers list them), one per line, in
 * buf (NUL-terminated, truncated to cap bytes); *len (may be NULL) receives
 * the full length without the NUL.  Launches nothing; for HBC_OP_ADJOINT it
 * builds the transposed tables if the plan has none yet (allocates). */
int hbc_plan_kernels(const hbc_plan* plan, int32_t op, char* buf, int64_t cap, int64_t* len);
/* Time `reps` applies captured in one HIP graph on `stream`; *ms receives the
 * mean milliseconds per apply (device events around the graph launch). */
int hbc_time_apply(const hbc_plan* plan, void* const* fields, int64_t nelem, int32_t nfields, int32_t reps,
                   void* stream, double* ms);

/* Capture `reps` calls of `plan` (op HBC_OP_APPLY: hbc_apply; HBC_OP_ADJOINT:
 * hbc_apply_adjoint), cycling over the `nfields` device fields (each of
 * `nelem` values), into one HIP graph on `stream` (not NULL), for replay
 * without per-launch overhead.  The fields and the plan must stay alive while
 * the graph exists.  A later change of the plan's launch shape
 * (hbc_plan_set_tune, hbc_plan_autotune) makes hbc_graph_launch return
 * HBC_EINVAL without launching: capture the graph again. */
#define HBC_OP_APPLY 0
#define HBC_OP_ADJOINT 1
typedef struct hbc_graph hbc_graph;
int hbc_graph_create(const hbc_plan* plan, int32_t op, void* const* fields, int64_t nelem, int32_t nfields,
                     int32_t reps, void* stream, hbc_graph** out);
int hbc_graph_launch(hbc_graph* g, void* stream);
void hbc_graph_destroy(hbc_graph* g);

/* ---- 27-point consumer (BC writes feed the inner operator, Sec. IV-C) -------- */
/* Plans from a Cartesian halo-1 program with inner == 1 and point layout.
 * x: ghosted field; y: data-only output, block by block, each block's data box
 * row-major.  y = 26 x_c - (sum of the 26 neighbours) per data cell. */
/* x_nelem / y_nelem must equal the field's cells and the data cell count. */
/* Unfused consumer: reads the ghosts already in x (run hbc_apply first). */
int hbc_stencil27(const hbc_plan* plan, const void* x, int64_t x_nelem, void* y, int64_t y_nelem, void* stream);
/* Fused: reads neighbours through the BC (copy from the source block or zero)
 * in one kernel; with write_ghosts != 0 it also writes x's covered ghost cells
 * (as hbc_apply would), otherwise x is only read (the ghosts are consumed
 * without being stored, Sec. IV-C's removal of BC writes no later reader
 * needs).  Each of a block's 26 ghost regions must be wholly one translated
 * copy of a neighbouring block, wholly zero rows, or wholly uncovered (read
 * from x as it is), and the plan must have no data rows; HBC_EUNSUPPORTED
 * otherwise (the unfused form has no such condition).  Blocks whose 32-plane
 * chunks reach 2 GiB are refused by both forms (HBC_EUNSUPPORTED). */
int hbc_fused_stencil27(const hbc_plan* plan, void* x, int64_t x_nelem, void* y, int64_t y_nelem,
                        int32_t write_ghosts, void* stream);

/* ---- consumer of the BC's ghosts: a stencil fused with the BC (Sec. IV-C) ----- */
/* Sec. IV-C: the boundary writes exist to feed the computation that follows,
 * and the two are optimised together.  The consumer here is a stencil of
 * offsets and weights: y[c, l] = sum_o weights[o] * x'[c + offsets[o], l] for
 * every data cell c of every block, where x' is the field after hbc_apply of
 * the plan.  offsets: noffsets x ndim positions of the global box (multiples
 * of the grid's step), 1 <= noffsets <= 64; every read of every data cell must
 * stay in its block's full region (HBC_EINVAL).  Point-major plans without
 * data rows (HBC_EUNSUPPORTED otherwise).  The consumer keeps a pointer to the
 * plan, which must outlive it; it reads the plan's rows as compiled at
 * creation (later new sub-vector values need a new consumer).  On a plan
 * created HBC_PLAN_HOST_ONLY the consumer is compiled on the host only:
 * hbc_consumer_stats works, hbc_consumer_apply returns HBC_EINVAL. */
typedef struct hbc_consumer hbc_consumer;
int hbc_consumer_create(const hbc_plan* plan, int32_t noffsets, const int64_t* offsets, const double* weights,
                        hbc_consumer** out);
/* y: device, y_nelem = data cells x inner values (block by block, each block's
 * data box row-major, inner values contiguous per cell); x: the plan's field
 * (x_nelem = cells x inner).  Sums in offset order (first product, then FMAs),
 * except where the offsets lie on at most 3 lines along the last dimension
 * (equal in the others), each within +-1 along it, without repeats: then line
 * by line (lines in order of first appearance, each in ascending last
 * coordinate), in both forms.
 * fused = 0: every read from x, ghosts as stored (run hbc_apply first).
 * fused = 1: reads of covered ghosts go through the BC: each cell whose
 * stencil reaches ghosts has one row composed at creation, entries (source
 * cell, weight x BC weight, the ghost row's component rotation) in offset
 * order then BC entry order, plus the weighted b; x is only read (its covered
 * ghosts are not; uncovered ghosts are read as stored). */
int hbc_consumer_apply(const hbc_consumer* c, const void* x, int64_t x_nelem, void* y, int64_t y_nelem,
                       int32_t fused, void* stream);
/* Cells whose stencil reaches a ghost (rows composed with the BC), and their entries. */
int hbc_consumer_stats(const hbc_consumer* c, int64_t* boundary_rows, int64_t* boundary_entries);
void hbc_consumer_destroy(hbc_consumer* c);

/* ---- FP64 interpolation weights on the device (setup, not part of an apply) -- */
/* For ghost layer k < h and tangential index t < N of any cubed-sphere face
 * side: base_dev[k*N + t] = first node, w_dev[(k*N + t)*4 + m] = weight of node
 * base + m, in the neighbour's tangential index counted in the direction of
 * the ghost face's tangential index.  Device arrays of h*N and 4*h*N. */
int hbc_cs_lagrange_weights(int64_t N, int64_t h, int32_t* base_dev, double* w_dev, void* stream);

/* ---- batched persistent apply (Sec. V-C: specialise once, run many) ---------- */
/* Concatenate the plans' work into one tile list (plans stay owned by the caller
 * and must outlive the batch; all plans need the same dtype and layout order). */
int hbc_batch_create(hbc_plan* const* plans, int32_t n, hbc_batch** out);
void hbc_batch_destroy(hbc_batch* b);
/* Bind one device field per plan (synchronous upload of the pointer table);
 * nelem[k] must equal plan k's cells * inner. */
int hbc_batch_bind(hbc_batch* b, void* const* fields, const int64_t* nelem);
/* One persistent launch applying every plan to its bound field. */
int hbc_batch_apply(hbc_batch* b, void* stream);
/* Capture one hbc_batch_apply into a HIP graph (re-captured on each call), then
 * hbc_batch_graph_launch replays it.  hbc_batch_set_tune and
 * hbc_batch_autotune drop the captured graph (the tile table it points at is
 * replaced): hbc_batch_graph_launch then returns HBC_EINVAL until the next
 * capture. */
int hbc_batch_graph_capture(hbc_batch* b, void* stream);
int hbc_batch_graph_launch(hbc_batch* b, void* stream);
/* Launch shape of the batch: block, lanes_per_row (0: each plan's own, else a
 * cap), rows_per_tile (inner values per tile; 0: one batch of rows per row
 * group, so a workgroup issues all its loads before its first store),
 * persistent workgroups. */
int hbc_batch_get_tune(const hbc_batch* b, hbc_tune* out);
int hbc_batch_set_tune(hbc_batch* b, const hbc_tune* t);
/* Try candidate launch shapes on the bound fields, keep the fastest; when
 * cache_path is not NULL, read / write the choice there (JSON lines keyed by
 * device, dtype, layout and work size).  *ms receives the best time per apply. */
int hbc_batch_autotune(hbc_batch* b, const char* cache_path, void* stream, double* ms);
int hbc_batch_stats(const hbc_batch* b, hbc_stats* out);

#ifdef __cplusplus
}
#endif

#endif /* HBC_H */
