// mesh.hpp -- host-side mesh plan (validation, device order, task tables).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/agile.h"
#include "agile_internal.hpp"

namespace agile {

struct PlanInput {
    int base[3];
    int max_level;
};

struct Plan {
    int64_t n = 0;
    int levels = 0;                         // finest level present
    std::vector<int> order;                 // device index -> caller index
    std::vector<int> perm;                  // caller index -> device index
    std::vector<BlockDesc> desc;            // device order
    std::vector<RestrictTask> restrict_tasks;
    std::vector<std::vector<ProlongTask>> prolong;  // [level] tasks filling level-l ghosts
    std::vector<char> prolong_dep;          // [level] some task reads a slab prolonged on level - 1
    std::vector<RefluxTask> reflux;
    int nhalo = 0;                          // ghost slabs at level jumps
    int nfreg = 0;                          // flux registers
    std::string error;
};

// Validate the leaf set and build the tables.  Returns AGILE_OK or
// AGILE_EINVAL (message in P.error).
int build_plan(const PlanInput &in, int64_t n, const agile_block_desc *blocks, Plan &P);

// Device bytes a mesh with this plan needs (state, ghosts, registers, tables).
size_t plan_device_bytes(const Plan &P, int nvar);

} // namespace agile
