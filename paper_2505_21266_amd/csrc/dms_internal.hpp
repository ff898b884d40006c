// dms_internal.hpp -- launch helpers shared by the single-field entry points
// and the batched plan.
#pragma once
#include "dms_common.hpp"

namespace dms {

// Largest number of fields in one batch (their tables live in LDS).
constexpr int kMaxBatchFields = 1024;

// One field of a batch: dims (x, y, z) and its offset in the concatenated
// arrays (values, orders and records alike).
struct BatchField {
    int64_t n[3];
    int64_t off;
};

// Gradient tile shapes (x extent; 1024 vertices per tile): 64x16, 32x32, 16x64.
constexpr int kTileVertsPerBlock = 1024;
constexpr int kGradVariants = 3;
constexpr int kTileX[kGradVariants] = {64, 32, 16};

// Checks the device and fills its lower-star tables once (one
// synchronisation of s); later calls return at once.
int init_tables(hipStream_t s);
// Takes the current device's address of the allocation-free extraction's
// scratch array (once per device).
int init_critical_scratch();
// ws: gradient_workspace_size(owned vertices) bytes for the queue of
// general vertices, or null (every tile then pairs its own).
size_t gradient_workspace_size(int64_t owned);
// mark (may be null): one bit per box record, set for the records that hold
// a critical cell (zeroed here first).
int launch_gradient(int variant, const int32_t *order, const int64_t *dims, const int64_t *lo,
                    const int64_t *hi, uint32_t *rec, uint32_t *mark, char *ws, hipStream_t s);
// mark (may be null): as for launch_gradient, over the concatenated records.
int launch_gradient_batch(int variant, const int32_t *order, const BatchField *fields, int nfields,
                          const int64_t *tile_start, const uint16_t *tile_field, int64_t total_tiles,
                          int64_t total_verts, uint32_t *rec, uint32_t *mark, char *ws, hipStream_t s);

// Ranks of n 64-bit unsigned keys (rank[i] = position of key i in the
// ascending stable sort), with the order passes.
size_t rank_u64_workspace_size(int64_t n);
int launch_rank_u64(const uint64_t *keys, int64_t n, int32_t *rank, char *ws, uint32_t *flags,
                    hipStream_t s);

// Batched order: values of all fields concatenated (float32); the field of
// element i is the f with foff[f] <= i < foff[f + 1] (foff on the device).
size_t order_batch_workspace_size(int64_t n);
int launch_order_batch(const float *values, int64_t n, const int64_t *foff, int nfields,
                       int32_t *order, char *ws, uint32_t *flags, hipStream_t s);

// Positions of cells of one dimension (codes (maxv << 8) | local index) in
// the filtration order of Section 2.1: rank[i] = place of codes[i] among
// them.  A code naming no cell of the grid raises DMS_FLAG_BADCODE.
size_t cell_rank_workspace_size(int64_t count);
int launch_cell_ranks(const int64_t *codes, int64_t count, int dim, const int32_t *order, const int64_t *dims,
                      int32_t *rank, char *ws, uint32_t *flags, hipStream_t s);

// Batched extraction over concatenated whole-field records; mask: the
// critical mask launch_gradient_batch set (records it does not flag are
// not read).
size_t critical_batch_workspace_size(int64_t n, int nfields);
int launch_critical_batch(const uint32_t *rec, const uint32_t *mask, int64_t n, const int64_t *foff,
                          int nfields, const BatchField *fields, int64_t *const crit[4], const int64_t cap[4],
                          int64_t *counts, int64_t *offsets, char *ws, uint32_t *flags, hipStream_t s);

}  // namespace dms
