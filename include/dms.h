/*
 * dms.h -- C ABI of the MI355X discrete-gradient library (libdms.so).
 *
 * The library computes the first step of Discrete Morse Sandwich on the
 * Freudenthal triangulation of a 3D regular grid: the global vertex order,
 * Robins et al.'s ProcessLowerStars discrete gradient, and the critical
 * simplices, plus the backward scatter of the differentiable D0 form and the
 * host-side D0 pairing that feeds it.
 *
 * Conventions shared by every call
 *  - Grids are C-ordered with x fastest: vertex (i, j, k) of a grid of
 *    dims = {nx, ny, nz} has id i + nx*(j + ny*k) ("offset in memory",
 *    Section 2.1).  dims, lo and hi are HOST arrays of three int64 (x, y, z).
 *  - The processed ("owned") box is the half-open [lo, hi); vertices of the
 *    grid outside it are ghosts (Section 2.2): read, never processed.
 *  - Array arguments are DEVICE pointers owned by the caller unless marked
 *    [host].  The calls of the path (order, gradient, extraction, backward,
 *    pairings' device halves) never allocate, free or synchronise; they
 *    enqueue work on `stream` (a hipStream_t, NULL = the default stream) and
 *    return.  Device set-up is explicit: dms_init, once per device, before
 *    the first gradient call on it; dms_batch_create calls it itself.
 *  - Argument errors are returned synchronously as a dms_status and nothing
 *    is enqueued; argument checks come before any device query, so they need
 *    no GPU.  A call that would launch work returns DMS_E_UNSUPPORTED when
 *    the current device is not a gfx950 (or there is no device), and the
 *    gradient calls return DMS_E_NOT_INITIALISED before dms_init succeeded
 *    on the current device.  Data-dependent conditions found on the device
 *    are OR-ed into *dev_flags (a device uint32 the caller zeroes), read
 *    after a sync.
 *  - Workspaces are caller-owned device buffers of at least the size the
 *    matching *_workspace_size call returns; their contents on entry are
 *    ignored.
 */
#ifndef DMS_H
#define DMS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DMS_OK = 0,
    DMS_E_ARG = 1,         /* null pointer, dims < 1, box outside the grid, bad dtype */
    DMS_E_SIZE = 2,        /* n > 2^31 - 1 vertices: int32 orders cannot rank them */
    DMS_E_WORKSPACE = 3,   /* workspace pointer null or smaller than required */
    DMS_E_UNSUPPORTED = 4, /* the current device is not a gfx950, or there is no device */
    DMS_E_HIP = 5,         /* a HIP runtime call (launch) failed */
    DMS_E_NOT_INITIALISED = 6 /* a gradient call before dms_init on the current device */
} dms_status;

/* bits OR-ed into *dev_flags by the device */
enum {
    DMS_FLAG_NAN = 1u,      /* a NaN value: the order (and all that follows) is undefined */
    DMS_FLAG_CAPACITY = 2u, /* a critical list exceeded its capacity; counts stay exact */
    DMS_FLAG_BADCODE = 4u   /* a cell code names no cell of the grid (dms_critical_sort) */
};

/* value types */
enum { DMS_F32 = 0, DMS_F64 = 1 };

/* Human-readable name of a status code (static string). */
const char *dms_status_str(int status);

/* Library version string (static). */
const char *dms_version(void);

/*
 * Device set-up for the current device -- the tabulated lower stars of
 * Section 2.3: a vertex whose lower neighbours are one member of each
 * opposite neighbour pair, or one of each but for a single pair with no or
 * both members lower, has its record looked up instead of running Robins'
 * pairing; the tables are filled once, by the same pairing code, on
 * `stream`.  Checks that the current device is a gfx950 (else
 * DMS_E_UNSUPPORTED), allocates the tables (held until the process ends),
 * fills them and synchronises `stream` once.  Idempotent per device and
 * safe to call from several threads.  Errors: DMS_E_UNSUPPORTED, DMS_E_HIP.
 */
int dms_init(void *stream);

/*
 * Copies the library's compile-time Kuhn star tables to [host] arrays:
 * nb[14*3] (dx, dy, dz) of each neighbour in linear-offset order,
 * tri[36*2], tet[24*3] (neighbour indices, ascending), edge_tris[14*6]
 * (-1 padded) and tri_tets[36*2].  Section 2.1 (Freudenthal triangulation;
 * the diagonal +(1,1,1) is this library's reading).  Returns DMS_OK.
 */
int dms_star_tables(int32_t *nb, int32_t *tri, int32_t *tet, int32_t *edge_tris, int32_t *tri_tets);

/* ----------------------------------------------------------------------------
 * Global vertex order -- Section 2.1 (injectivity by pre-sorting vertices by
 * value, ties broken by offset in memory) and Section 3 (Array
 * Preconditioning).
 *
 * order[v] = number of vertices w with (f(w), w) < (f(v), v), where -0.0 and
 * +0.0 compare equal and +-inf are ordered normally.  values: n float32
 * (dtype DMS_F32) or float64 (DMS_F64); order: n int32.  A NaN sets
 * DMS_FLAG_NAN and leaves order undefined.
 * Errors: DMS_E_ARG (null pointer, n < 0, bad dtype), DMS_E_SIZE
 * (n > 2^31 - 1), DMS_E_WORKSPACE, DMS_E_HIP.
 * -------------------------------------------------------------------------- */
size_t dms_order_workspace_size(int64_t n, int dtype);
int dms_order(const void *values, int dtype, int64_t n, int32_t *order, void *workspace,
              size_t workspace_bytes, uint32_t *dev_flags, void *stream);

/* ----------------------------------------------------------------------------
 * Discrete gradient -- Section 2.3 (discrete vectors; the gradient algorithm
 * of Robins et al., one lower star per vertex) with the lexicographic
 * simplex comparison of Section 2.1.
 *
 * For every vertex x of the box [lo, hi), pairs the cells of its lower star
 * (x and the simplices of its star whose other vertices precede x in
 * `order`) with Robins' ProcessLowerStars and writes one 128-bit record
 * (four uint32, little-endian bit numbering) to rec[4 * r], r = box index
 * with x fastest:
 *   bits [4e, 4e+4), e = 0..13: neighbour edge e -- 0 not in L(x),
 *     1 paired with x, 2 critical, 3+j paired with the j-th star triangle
 *     containing e (ascending triangle index);
 *   bits [56+2t, 58+2t), t = 0..35: star triangle t -- 0 not paired with a
 *     tet, 1+j paired with the j-th star tet containing t.
 * Every other cell state follows: x is critical iff all edge fields are 0; a
 * triangle is in L(x) iff both its edges are, a head iff an edge field names
 * it, critical if in L(x), not a head and not a tail; a tet is in L(x) iff
 * its three edges are, critical unless a triangle field names it.
 * order: int32 of the whole grid (dims), a permutation of 0..n-1 or any
 * injective int32 labelling with the same relative order (values must be
 * < 2^31 - 1).  An empty box is allowed and enqueues nothing.
 * workspace: dms_gradient_workspace_size(dims, lo, hi) bytes (about one
 * byte per box vertex) holding a queue through which vertices whose lower
 * star needs the full pairing loop are gathered and paired in dense waves;
 * or NULL (with workspace_bytes 0), in which case they are paired where
 * they are found -- the same records, slower on smooth fields.
 * critical_mask: NULL, or ceil(nbox / 32) device uint32 (nbox = vertices of
 * the box) that receive one bit per record in box order, bit r % 32 of word
 * r / 32 set iff L(x) of record r holds a critical cell; every word is
 * written.  dms_critical_simplices reads only the records it flags.
 * Errors: DMS_E_ARG (null order/rec, dims < 1, box outside the grid),
 * DMS_E_SIZE, DMS_E_WORKSPACE (non-null workspace below the size), DMS_E_HIP.
 * -------------------------------------------------------------------------- */
size_t dms_gradient_workspace_size(const int64_t dims[3], const int64_t lo[3], const int64_t hi[3]);
int dms_discrete_gradient(const int32_t *order, const int64_t dims[3], const int64_t lo[3],
                          const int64_t hi[3], uint32_t *rec, uint32_t *critical_mask, void *workspace,
                          size_t workspace_bytes, void *stream);

/* ----------------------------------------------------------------------------
 * Discrete gradient from the values -- the same lower stars, with x and its
 * neighbours compared by (value, vertex id) directly, as Section 2.1 defines
 * the order (-0.0 equal to +0.0), instead of through the ranks of the global
 * order.  Needs no sort (a step the paper's Array Preconditioning performs
 * once, Section 3), so a block of a larger field can be processed from its
 * values and ghost layer alone.  The records equal those of
 * dms_discrete_gradient on the order of the same values, bit for bit.
 * values: DMS_F32 or DMS_F64 array of the whole grid (dims), device.
 * dev_flags: DMS_FLAG_NAN is OR-ed in when a value read is NaN (the records
 * are then undefined).  Other arguments as for dms_discrete_gradient.
 * Errors: DMS_E_ARG (bad dtype, null values/rec/dev_flags, dims < 1, box
 * outside the grid), DMS_E_SIZE, DMS_E_WORKSPACE, DMS_E_HIP.
 * -------------------------------------------------------------------------- */
int dms_discrete_gradient_values(const void *values, int dtype, const int64_t dims[3],
                                 const int64_t lo[3], const int64_t hi[3], uint32_t *rec,
                                 uint32_t *critical_mask, void *workspace, size_t workspace_bytes,
                                 uint32_t *dev_flags, void *stream);

/* ----------------------------------------------------------------------------
 * Critical simplices -- Section 2.6 (zero-persistence skip: every
 * non-critical simplex forms a zero-persistence pair with its vector
 * partner, so only critical simplices go on) and Section 3 (Extract).
 *
 * Decodes the records of box [lo, hi) (as written by dms_discrete_gradient
 * with the same dims and box) and writes, per dimension d = 0..3, the
 * critical cells as int64 codes (max_vertex_id << 8) | local, where local is
 * the cell's index in its max vertex's star table of that dimension (0 for
 * the vertex itself, the neighbour edge 0..13, star triangle 0..35, star
 * tet 0..23), listed by increasing code.  crit0..crit3: device arrays with
 * room for cap[d] codes ([host] cap); counts: 4 device int64, always the
 * exact totals.  When a total exceeds its capacity the list is truncated
 * and DMS_FLAG_CAPACITY is set.
 * critical_mask: NULL (every record is read), or the mask the gradient call
 * wrote with these records: only records whose bit is set are read, the
 * others count as holding no critical cell (Section 2.6: most vertices hold
 * none, so the extraction then reads about 1/128 of the record bytes).  A
 * mask from other records gives undefined lists.
 * Errors: DMS_E_ARG, DMS_E_SIZE, DMS_E_WORKSPACE, DMS_E_HIP.
 * -------------------------------------------------------------------------- */
size_t dms_critical_workspace_size(const int64_t dims[3], const int64_t lo[3], const int64_t hi[3]);
int dms_critical_simplices(const uint32_t *rec, const uint32_t *critical_mask, const int64_t dims[3],
                           const int64_t lo[3], const int64_t hi[3], int64_t *crit0, int64_t *crit1,
                           int64_t *crit2, int64_t *crit3, const int64_t cap[4], int64_t *counts,
                           void *workspace, size_t workspace_bytes, uint32_t *dev_flags, void *stream);

/* ----------------------------------------------------------------------------
 * The same extraction with no workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  The workspace is a device
 * array inside the library, one per GPU, held until the process ends:
 * about 16.4 MB, enough for boxes of up to 160 * 1024 tiles of 1024
 * records (167,772,160 vertices).  It never allocates or frees memory; the
 * array's address on the current device is taken by dms_init.  Calls on one
 * GPU share that array: two calls that overlap in time on one GPU (on
 * different streams) race and give undefined lists; calls in one stream's
 * order do not.  Every word the kernels read is first written by the same
 * call, so nothing carries over from an earlier call.  Arguments as for
 * dms_critical_simplices.
 * Errors: DMS_E_ARG, DMS_E_SIZE (box beyond the limit above, or a grid
 * beyond 2^40 vertices), DMS_E_UNSUPPORTED, DMS_E_NOT_INITIALISED (dms_init
 * has not run on the current device), DMS_E_HIP.
 * -------------------------------------------------------------------------- */
int dms_critical_simplices_noalloc(const uint32_t *rec, const uint32_t *critical_mask,
                                   const int64_t dims[3], const int64_t lo[3], const int64_t hi[3],
                                   int64_t *crit0, int64_t *crit1, int64_t *crit2, int64_t *crit3,
                                   const int64_t cap[4], int64_t *counts, uint32_t *dev_flags,
                                   void *stream);

/* ----------------------------------------------------------------------------
 * Values of simplices -- Section 2.5: a persistence pair is embedded at
 * (f(birth simplex), f(death simplex)), where f of a simplex is the value of
 * its highest vertex.  out[i] = values[codes[i] >> 8] as float64 (codes as
 * dms_critical_simplices writes them; values DMS_F32 or DMS_F64, n
 * entries).  A code naming a vertex outside [0, n) gives NaN.
 * Errors: DMS_E_ARG (bad dtype, null pointer with count > 0), DMS_E_HIP.
 * -------------------------------------------------------------------------- */
int dms_simplex_values(const void *values, int dtype, int64_t n, const int64_t *codes, int64_t count,
                       double *out, void *stream);

/* ----------------------------------------------------------------------------
 * Backward of the birth/death values (D0 or D2 pairs) -- Section 2.5: f of a
 * simplex is its highest vertex value, so d(birth)/d(f) and d(death)/d(f)
 * are indicator vectors at the max vertex of each simplex.
 *
 * grad[v] = sum over pairs p with maxv(birth_code[p]) == v of g_birth[p]
 *         + sum over pairs p with maxv(death_code[p]) == v of g_death[p],
 * where maxv(code) = code >> 8.  grad (n float64) is overwritten.  The sum
 * is deterministic: each vertex adds its contributions in one fixed order
 * (the births in pair order, then the deaths in pair order), after a stable
 * sort of the 2 * npairs contributions by vertex; no atomics.  Codes naming
 * vertices outside [0, n) are ignored.
 * workspace: dms_gradient_backward_workspace_size(npairs) bytes.
 * Errors: DMS_E_ARG (null pointer with npairs > 0 or n > 0, npairs over
 * 2^30), DMS_E_WORKSPACE, DMS_E_UNSUPPORTED, DMS_E_HIP.
 * -------------------------------------------------------------------------- */
size_t dms_gradient_backward_workspace_size(int64_t npairs);
int dms_gradient_backward(const int64_t *birth_code, const int64_t *death_code,
                          const double *g_birth, const double *g_death, int64_t npairs,
                          double *grad, int64_t n, void *workspace, size_t workspace_bytes,
                          void *stream);

/* ----------------------------------------------------------------------------
 * D0 pairing on the host -- Section 2.6 and Algorithm 1 (PairExtremaSaddles).
 *
 * From whole-grid records ([host] rec, 4 uint32 per vertex of dims, box =
 * whole grid), the [host] order and the [host] list of critical edge codes,
 * builds the extremum graph (each critical edge descends from both vertices
 * along the vertex-edge vectors to a minimum; triplets with two distinct
 * minima are kept), visits the triplets by increasing edge (Section 2.1
 * comparison) and pairs each edge with the younger of its two
 * representatives.  Writes up to `capacity` pairs to [host] pair_edge
 * (edge codes) and pair_min (vertex ids) in processing order and their count
 * to *npairs.  Errors: DMS_E_ARG (null pointer, code out of range),
 * DMS_E_WORKSPACE (capacity too small: *npairs holds the count needed).
 * -------------------------------------------------------------------------- */
int dms_d0_pairs_host(const uint32_t *rec, const int32_t *order, const int64_t dims[3],
                      const int64_t *crit1, int64_t n1, int64_t *pair_edge, int64_t *pair_min,
                      int64_t capacity, int64_t *npairs);

/* ----------------------------------------------------------------------------
 * Batched form: many float32 fields of uneven shapes (ensemble members, time
 * steps) through order, gradient and extraction in one graph launch.  Each
 * field is processed exactly as the single-field calls would process it
 * with box = the whole field (Sections 2.1, 2.3, 2.6); the batch only shares
 * launches.
 *
 * dms_batch_create: dims = [host] 3 * nfields sides (x, y, z) of the fields,
 * in order; dtype must be DMS_F32.  tune != 0 times the gradient tile
 * shapes on the first run (that run synchronises) unless tune_cache (a file
 * path, may be NULL) already holds a choice for these shapes; the choice is
 * appended to tune_cache.  Allocates small device tables and a private
 * capture stream; returns DMS_E_ARG, DMS_E_SIZE (over 1024 fields or more
 * than 2^31 - 1 vertices in all), DMS_E_UNSUPPORTED (dtype), DMS_E_HIP.
 *
 * dms_batch_run: values = all fields concatenated in order (field f starts at
 * off[f] = sum of the vertex counts of the fields before it), device float32;
 * order (int32) and rec (4 uint32 per vertex) are concatenated the same way
 * and hold each field's own order and records.  crit0..crit3 receive, per
 * dimension, the critical cells of all fields, field after field, as
 * (field-local vertex id << 8) | local index; cap[4] [host] are their
 * capacities.  counts (device, 4 * nfields int64) receives counts[4 f + d];
 * offsets (device, 4 * (nfields + 1) int64) receives the first slot of field
 * f in list d at offsets[d * (nfields + 1) + f], and the total at f = nfields.
 * The first run (and any run whose pointers or capacities differ from the
 * previous one) records the launches into a hipGraph; the others replay it
 * on `stream`.  dev_flags as for the single-field calls.
 * ------------------------------------------------------------------------- */
typedef struct dms_batch dms_batch;
int dms_batch_create(const int64_t *dims, int nfields, int dtype, int tune, const char *tune_cache,
                     dms_batch **out);
size_t dms_batch_workspace_size(const dms_batch *batch);
int64_t dms_batch_total(const dms_batch *batch);   /* vertices in all fields */
int dms_batch_variant(const dms_batch *batch);     /* chosen gradient tile shape: 0 64x16, 1 32x32, 2 16x64 */
int dms_batch_run(dms_batch *batch, const void *values, int32_t *order, uint32_t *rec, int64_t *crit0,
                  int64_t *crit1, int64_t *crit2, int64_t *crit3, const int64_t cap[4],
                  int64_t *counts, int64_t *offsets, void *workspace, size_t workspace_bytes,
                  uint32_t *dev_flags, void *stream);
void dms_batch_destroy(dms_batch *batch);

/* ----------------------------------------------------------------------------
 * D0 pairing on the GPU, extremum-graph half -- Section 2.6 (for each
 * critical edge, the minima reached by descending from its two vertices along
 * the vertex-edge vectors) and the visiting order of Algorithm 1 (increasing
 * edge, Section 2.1 comparison).
 *
 * rec: the records of the WHOLE grid (dms_discrete_gradient with the box equal
 * to the grid); order: the grid's order; crit0 / crit1: its critical vertex
 * and edge codes (dms_critical_simplices).  All device arrays.
 * Outputs (device): tri_edge, tri_min0, tri_min1 [capacity n1]: the triplets
 * whose two minima differ, sorted by edge; tri_min* are indices into crit0
 * (the minimum reached from the edge's higher vertex first); min_order[n0]:
 * the order of each minimum; *ntri: the number of triplets (int64).
 * workspace: dms_d0_workspace_size(dims, n1) bytes.  A minimum missing from
 * crit0 (a truncated list) sets DMS_FLAG_CAPACITY in *dev_flags.
 * Errors: DMS_E_ARG, DMS_E_SIZE, DMS_E_WORKSPACE, DMS_E_HIP.
 * -------------------------------------------------------------------------- */
size_t dms_d0_workspace_size(const int64_t dims[3], int64_t n1);
int dms_d0_triplets(const uint32_t *rec, const int32_t *order, const int64_t dims[3],
                    const int64_t *crit0, int64_t n0, const int64_t *crit1, int64_t n1,
                    int64_t *tri_edge, int32_t *tri_min0, int32_t *tri_min1, int32_t *min_order,
                    int64_t *ntri, void *workspace, size_t workspace_bytes, uint32_t *dev_flags,
                    void *stream);

/* ----------------------------------------------------------------------------
 * D0 pairing, union-find half -- Algorithm 1 (PairExtremaSaddles) over the
 * sorted triplets of dms_d0_triplets, on [host] arrays: each triplet joins
 * the classes of its minima; the younger representative (higher order) dies
 * at the edge.  Outputs pair_edge (edge codes) and pair_min (indices into
 * crit0) in visiting order, up to capacity; *npairs is the exact count.
 * Errors: DMS_E_ARG (bad arguments or a minimum index outside [0, n0)),
 * DMS_E_WORKSPACE (more pairs than capacity; npairs is still exact).
 * -------------------------------------------------------------------------- */
int dms_d0_pairs_sorted_host(const int64_t *tri_edge, const int32_t *tri_min0, const int32_t *tri_min1,
                             int64_t ntri, const int32_t *min_order, int64_t n0, int64_t *pair_edge,
                             int32_t *pair_min, int64_t capacity, int64_t *npairs);

/* ----------------------------------------------------------------------------
 * Critical cells in filtration order -- Section 2.1 (a cell's key is the list
 * of its vertex orders sorted decreasingly; cells of one dimension compare by
 * their keys lexicographically) and the local sort of the extracted lists
 * (Section 3, Extract).
 *
 * codes [device, count]: cells of dimension dim (0..3) of the grid dims, as
 * dms_critical_simplices writes them, (maxv << 8) | local index, in any
 * order.  order [device]: the grid's order (dms_order).  sorted [device,
 * count]: receives the same codes in increasing filtration order (unique:
 * distinct cells have distinct keys); it must not overlap codes.
 * workspace: dms_critical_sort_workspace_size(count) bytes.  A code naming no
 * cell of the grid sets DMS_FLAG_BADCODE in *dev_flags (such cells sort last).
 * Errors: DMS_E_ARG, DMS_E_SIZE (count above 2^31 - 1), DMS_E_WORKSPACE,
 * DMS_E_HIP.
 * -------------------------------------------------------------------------- */
size_t dms_critical_sort_workspace_size(int64_t count);
int dms_critical_sort(const int64_t *codes, int64_t count, int dim, const int32_t *order,
                      const int64_t dims[3], int64_t *sorted, void *workspace, size_t workspace_bytes,
                      uint32_t *dev_flags, void *stream);

/* ----------------------------------------------------------------------------
 * D2 pairing on the GPU, extremum-graph half -- Section 2.6 (D2 is computed
 * like D0 on the dual complex, where every discrete vector is reversed).  The
 * dual graph has one node per tet and one for the outside of the grid; a
 * triangle on the grid boundary joins its one tet to the outside node.  From
 * the two cofacet tets of each critical triangle the dual v-path is followed
 * (a tet that is the head of a gradient pair continues through its tail
 * triangle into the other tet containing it) to a critical tet or the outside.
 *
 * rec: the records of the WHOLE grid; order: the grid's order; crit2 / crit3:
 * its critical triangle and tet codes as dms_critical_simplices lists them
 * (crit3 in increasing code order).  All device arrays.
 * Outputs (device): tri_code, tri_max0, tri_max1 [capacity n2]: the triplets
 * whose two maxima differ, by DECREASING triangle (Section 2.1 order);
 * tri_max* are indices into crit3, n3 standing for the outside node;
 * max_rank[n3]: the place of each critical tet in the Section 2.1 order of
 * crit3; *ntri: the number of triplets (int64).
 * workspace: dms_d2_workspace_size(n2, n3) bytes.  A maximum missing from
 * crit3 (a truncated list) or a bad code sets DMS_FLAG_CAPACITY.
 * Errors: DMS_E_ARG, DMS_E_SIZE, DMS_E_WORKSPACE, DMS_E_HIP.
 * -------------------------------------------------------------------------- */
size_t dms_d2_workspace_size(int64_t n2, int64_t n3);
int dms_d2_triplets(const uint32_t *rec, const int32_t *order, const int64_t dims[3],
                    const int64_t *crit2, int64_t n2, const int64_t *crit3, int64_t n3,
                    int64_t *tri_code, int32_t *tri_max0, int32_t *tri_max1, int32_t *max_rank,
                    int64_t *ntri, void *workspace, size_t workspace_bytes, uint32_t *dev_flags,
                    void *stream);

/* ----------------------------------------------------------------------------
 * D2 pairing, union-find half -- the dual of Algorithm 1 over the triplets
 * of dms_d2_triplets, on [host] arrays, in their (decreasing) order: each
 * triplet joins the classes of its maxima; the lower representative (smaller
 * max_rank; index n3, the outside node, is above every tet) dies at the
 * triangle.  Outputs pair_tri (triangle codes) and pair_max (indices into
 * crit3) in visiting order, up to capacity; *npairs is the exact count.
 * Errors: DMS_E_ARG (bad arguments or a maximum index outside [0, n3]),
 * DMS_E_WORKSPACE (more pairs than capacity; npairs is still exact).
 * -------------------------------------------------------------------------- */
int dms_d2_pairs_sorted_host(const int64_t *tri_code, const int32_t *tri_max0, const int32_t *tri_max1,
                             int64_t ntri, const int32_t *max_rank, int64_t n3, int64_t *pair_tri,
                             int32_t *pair_max, int64_t capacity, int64_t *npairs);

#ifdef __cplusplus
}
#endif

#endif /* DMS_H */
