// Host-side internals shared by the driver (lmbd_api.hip) and the serving
// runtime (lmbd_serve.hip).  Not part of the public ABI.
#pragma once

#include "lmbd.h"
#include "lmbd_internal.h"

#include <vector>

namespace lmbd {

// Neighbour counts of one structure as the device will find them.
struct StructCounts {
    std::vector<Counts> cnt;
    int n_cells = 0;
    bool forces = false;
};

// Validate one structure (host arrays) and count its neighbourhoods.
lmbd_status analyse_structure(const lmbd_params* params, const lmbd_structure& s, StructCounts& out);

// Exact device bytes of one lmbd_compute_batch call on the structures whose
// counts are given, in this order, with a species table of n_species entries.
lmbd_status layout_bytes(const lmbd_params* params, int n_species, const std::vector<const StructCounts*>& parts,
                         size_t* bytes);

// Make every later call of the context carve its buffers from [base, base +
// bytes) (device memory owned by the caller) instead of allocating; NULL
// returns the context to its own cached allocations.
void set_workspace(lmbd_context* ctx, void* base, size_t bytes);

}  // namespace lmbd
