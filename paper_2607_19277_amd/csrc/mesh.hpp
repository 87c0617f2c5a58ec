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

// Where a block of a regridded mesh takes its data from (old caller indices).
struct RegridSource {
    int kind = 0;        // 0 copy of src[0], 1 child `octant` of parent src[0], 2 mean of children src[0..7]
    int octant = 0;      // x + 2 y + 4 z of the child inside its parent
    int src[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
};

// Refine / coarsen decision from a per-block error: leaves above `refine`
// below `max_level` are refined; complete octets of leaves (level >= 2) all
// below `coarsen` and none refined are coarsened; refinement is propagated
// to coarser face neighbours and coarsening withdrawn until 2:1 balance holds
// across faces.  One level of change per leaf; periodic domain.  The new
// leaves come sorted by (level, x, y, z), each with its data source.
int regrid_decide(const PlanInput &in, int64_t n, const agile_block_desc *blocks, const double *err, int max_level,
                  double refine, double coarsen, std::vector<agile_block_desc> &out, std::vector<RegridSource> &src,
                  int64_t &refined, int64_t &coarsened, std::string &error);

// Data sources of the blocks nw of a regridded mesh from the blocks old, by
// position (copy, child of an old parent, or mean of 8 old children).
int regrid_sources(const std::vector<agile_block_desc> &old, const std::vector<agile_block_desc> &nw,
                   std::vector<RegridSource> &src, std::string &error);

} // namespace agile
