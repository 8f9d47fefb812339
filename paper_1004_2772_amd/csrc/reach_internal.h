// Device view of a model and helpers shared by the reachability units.
#pragma once

#include <vector>

#include "internal.h"

// Packed transition table [P][L][K] of uint2:
//   x = target | guard_var << 16 | eff_var << 24   (0xFF = none)
//   y = guard_val | eff_val << 16
struct ModelView {
    const uint2 *trans;
    uint32_t P, L, S, K, W;
    uint32_t magic_PK;   // ceil(2^32 / (P*K)) for __umulhi division
    uint32_t magic_K;
};

namespace lhs {

lhs_status validate_model(const reach_model *m);
void pack_model(const reach_model *m, std::vector<uint2> &out);
ModelView model_view(const reach_model *m, const uint2 *d_trans);
size_t expand_lds_bytes(uint32_t W, uint32_t tcap);
lhs_status ensure_bfs_buffers(lhs_table *t);
uint64_t auto_capacity(const reach_model *m);

}  // namespace lhs
