// noalloc.hip -- device scratch of the regrid entry point that allocates no
// device memory (agile_mesh_regrid_noalloc).
//
// The remap task table of such a regrid lives in one file-scope device array
// of AGILE_NOALLOC_MAX_BLOCKS records, which every GPU the library runs on
// holds until the process ends.  Host code never passes the array's name to a
// kernel or a copy (on the host that name is only a stand-in): its device
// address is looked up once per device with hipGetSymbolAddress, with that
// device current, and kept.  Every call on a GPU shares that GPU's array, so
// two such calls that overlap on one GPU race; each call writes the records
// it reads before its kernel runs, so nothing needs clearing.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/agile.h"
#include "agile_internal.hpp"

namespace agile {

namespace {

static __device__ __align__(256) RemapTask scratch[AGILE_NOALLOC_MAX_BLOCKS];

std::mutex g_mu;
std::vector<RemapTask *> g_ptr;   // per device: the address of `scratch` there

} // namespace

// Device address of the scratch table on `device`, which must be the current
// device; looked up on the first call for that device.
RemapTask *noalloc_scratch(int device, std::string &err) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (device < 0) {
        err = "no current device";
        return nullptr;
    }
    if (int(g_ptr.size()) <= device) g_ptr.resize(size_t(device) + 1, nullptr);
    if (!g_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return nullptr;
        }
        g_ptr[device] = static_cast<RemapTask *>(p);
    }
    return g_ptr[device];
}

} // namespace agile
