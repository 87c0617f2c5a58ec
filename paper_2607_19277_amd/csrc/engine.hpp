// engine.hpp -- device block pool and step sequencing shared by the single-mesh
// API and the batched serving API.
//
// A pool holds the state of any number of meshes: each resident mesh owns a
// contiguous range of pool blocks (U, XE, per-block signal maxima,
// descriptors), a range of ghost slabs and flux registers, and one mesh slot
// (parameters, dt, time, reductions).  Its host plan is rewritten to pool
// indices on admission.  One step advances every active mesh with its own
// CFL dt: the kernels walk the concatenated task tables and an active-block
// list, so a batch of uneven meshes and levels is updated by one launch per
// kernel class.  The launch sequence of a step can be captured once into a
// hipGraph and replayed while the set of active meshes is unchanged.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/agile.h"
#include "agile_internal.hpp"
#include "mesh.hpp"

namespace agile {

hipError_t launch_stage(const StageArgs &a, int riemann, int precision, hipStream_t s);
hipError_t launch_restrict(const RestrictTask *t, int n, const double *U, double *halo, int NV, hipStream_t s);
// XE: the x-boundary copy of U, read for the coarse blocks' x-boundary
// columns, or null
hipError_t launch_prolong(const ProlongTask *t, int n, const BlockDesc *desc, const MeshParams *mp, const double *U,
                          const double *XE, double *halo, int NV, int srhd, hipStream_t s);
hipError_t launch_reflux(const RefluxTask *t, int n, MeshParams *mp, double *U, double *XE, const double *freg,
                         unsigned long long *smax, unsigned long long *cmax, int NV, double bw, int last,
                         hipStream_t s);
hipError_t launch_reflux_restrict(const RefluxTask *rt, int nref, const RestrictTask *st, int nres, MeshParams *mp,
                                  double *U, double *XE, const double *freg, double *halo, unsigned long long *smax,
                                  unsigned long long *cmax, int NV, double bw, int last, hipStream_t s);
hipError_t launch_xexport(const double *U, double *XE, int first, int n, int NV, hipStream_t s);
hipError_t launch_smax(const BlockDesc *desc, MeshParams *mp, const double *U, unsigned long long *smax,
                       unsigned long long *cmax, int first, int n, int NV, hipStream_t s);
hipError_t launch_mesh_reduce(MeshParams *mp, const int *meshes, int nmesh, const unsigned long long *smax,
                              const unsigned long long *cmax, int mode, hipStream_t s);
hipError_t launch_mhd_stage(const SweepArgs &a, int stage, int precision, hipStream_t s);
hipError_t launch_glm_decay(const BlockDesc *desc, MeshParams *mp, double *U, double *XE, const int *list,
                            int nblocks, double hfrac, hipStream_t s);
hipError_t launch_set_dt(MeshParams *mp, int mesh, double dt, hipStream_t s);
hipError_t launch_permute(const double *src, double *dst, const int *map, int first, int nblocks, int per_block,
                          int gather, hipStream_t s);
hipError_t launch_lohner(const BlockDesc *desc, const double *U, const double *halo, int first, int n, int NV, int v,
                         double eps, double *out, hipStream_t s);
hipError_t launch_remap(const RemapTask *t, int n, const BlockDesc *desc, const MeshParams *mp, const double *U,
                        const double *halo, int NV, int srhd, double *out, hipStream_t s);
hipError_t launch_read_ghosts(const BlockDesc *desc, const double *U, const double *halo, double *out, int first,
                              int n, int NV, hipStream_t s);
hipError_t launch_stream_copy(const void *src, void *dst, size_t bytes, hipStream_t s);
hipError_t launch_permute_tiles(const double *src, double *dst, const int *map, int first, int ntiles, int NV,
                                int te, int gather, hipStream_t s);

// host copies between a state in blocks of (16 te)^3 cells and 16^3 tiles:
// caller tile q is sub-tile q mod te^3 (x fastest) of block q / te^3 and sits
// at perm[q] of the tile array
void tiles_from_blocks(const double *blocks, double *tiles, const int *perm, int ntiles, int nv, int te);
void blocks_from_tiles(const double *tiles, double *blocks, const int *perm, int ntiles, int nv, int te);

// first-fit allocator of index ranges in [0, cap)
class RangeAlloc {
public:
    void reset(int cap);
    int alloc(int n);             // start index, or -1; n == 0 always succeeds with 0
    void release(int start, int n);
    bool can_alloc(int n) const;
    int free_total() const { return free_total_; }

private:
    std::map<int, int> free_;     // start -> length
    int free_total_ = 0;
};

struct EngineConfig {
    int physics = AGILE_EULER;
    int riemann = AGILE_HLLC;
    int precision = AGILE_FP64;
    int limiter = 0;              // reconstruction slope: 0 minmod, 1 van Leer
    int rk = 2;                   // SSP Runge-Kutta stages: 2 or 3
    hipStream_t stream = nullptr;
    int cap_blocks = 0;
    int cap_halo = 0;
    int cap_freg = 0;
    int cap_meshes = 1;
    void *pool = nullptr;         // caller-owned device memory to carve every array
    size_t pool_bytes = 0;        // from (null: the engine allocates its own)
};

// Device bytes an engine with config c occupies (carved from a caller's pool
// or allocated), the arrays 256-byte aligned.
size_t engine_device_bytes(const EngineConfig &c);

struct MeshSlot {
    bool used = false;
    bool active = false;          // advanced by step()
    agile_config cfg{};
    Plan plan;                    // tables rewritten to pool indices
    int first = 0, halo0 = 0, freg0 = 0;
    int *d_perm = nullptr;        // caller order -> local device order (inside the pool's array)
    int tile_edge = 1;            // 16^3 tiles per caller block edge (caller state layout)
    int64_t steps_target = -1;    // -1: unlimited
    int64_t steps_done = 0;
    uint64_t tag = 0;
};

class Engine {
public:
    ~Engine();
    int init(const EngineConfig &c, std::string &err);

    // Validate / size a block list for this engine (no device work).
    int plan(const agile_config &cfg, int64_t n, const agile_block_desc *b, Plan &P, std::string &err) const;
    bool fits(const Plan &P) const;
    // Admit a mesh with a prepared plan; the state is uploaded on the stream.
    // carry (may be null): simulated time, last dt and the non-physical flag
    // taken over from an earlier form of the same mesh (a regrid).
    // u_edge: u holds blocks of (16 u_edge)^3 cells, each the u_edge^3 tiles
    // of P in order (1: u is in 16^3 tiles); later readbacks use the layout
    // of slot_edge.
    int add(const agile_config &cfg, Plan &&P, const double *u, int u_on_device, int64_t steps, uint64_t tag,
            int *slot, std::string &err, const MeshParams *carry = nullptr, int u_edge = 1, int slot_edge = 1);
    int remove(int slot);
    int set_active(int slot, bool active);
    // steps already taken by the mesh in a slot (carried over a re-admission)
    int set_progress(int slot, int64_t steps_done);

    int step_cfl(int nsteps, std::string &err);         // every active mesh, CFL dt each
    int step_dt(int slot, double dt, std::string &err);  // one mesh (the only active one), given dt
    int fill_ghosts(std::string &err);                   // ghost slabs of every active mesh
    int read_state(int slot, double *out, int out_on_device, std::string &err);
    int read_ghosts(int slot, double *out, int out_on_device, std::string &err);
    // Loehner estimate of conserved variable v of a mesh (ghosts filled
    // first): per block, in the caller's block order, into host memory.
    int lohner(int slot, int v, double eps, double *out_host, std::string &err);
    // Data of a regridded mesh from this one: src in the caller's block
    // indices of `slot`, out a device array [src.size()][nvar][16^3].
    // d_tasks: device room for src.size() task records (null: allocated here).
    int remap(int slot, const std::vector<RegridSource> &src, double *out_dev, std::string &err,
              RemapTask *d_tasks = nullptr);
    // Whether a mesh with plan P fits once mesh `slot` has been removed.
    bool fits_replacing(int slot, const Plan &P) const;
    // The stage buffer U[1] as room for n blocks of state (its content is free
    // between steps), or null when the pool holds fewer blocks.
    double *stage_buffer(int64_t n) const { return n <= cfg_.cap_blocks ? U_[1] : nullptr; }
    int read_params(int slot, MeshParams &hp, std::string &err);
    // choose the stage shapes (kslab / xcd of the first and middle stages, and
    // of the last stage of a step): by timing whole steps on a copy of the
    // state, or, without room for the copy, single launches of each stage
    // kind on (at most max_blocks of) the active blocks
    int tune(std::string &err, int max_blocks = 4096);

    // kernel timing (eager launches only) of the kernel classes in the bit mask `kinds`
    int profile(int kinds, std::string &err);
    int profile_read(int kind, double &ms, int64_t &launches, std::string &err);

    const MeshSlot &slot(int s) const { return slots_[s]; }
    int nvar() const { return nvar_; }
    int nslots() const { return int(slots_.size()); }
    int active_blocks() const { return nlist_; }
    int cap_blocks() const { return cfg_.cap_blocks; }
    int cap_halo() const { return cfg_.cap_halo; }
    int cap_freg() const { return cfg_.cap_freg; }
    int free_blocks() const { return blocks_.free_total(); }
    hipStream_t stream() const { return cfg_.stream; }
    // solver template of the stage kernel: the Euler solvers, or 3 for the
    // SRHD module (local Lax-Friedrichs on (rho, Gamma v, p))
    int stage_solver() const { return cfg_.physics == AGILE_SRHD ? 3 : cfg_.riemann; }

    int tune_launches(std::string &err, int max_blocks);

    bool use_graph = false;
    // stage shape of the first and middle stages, and of the last stage of a
    // step (the stage that also reduces the signal rate).  Whole steps on
    // Sedov, KH 256^3 and the paper's numerics run as fast or faster (FP32
    // flux: 2%) with the plain workgroup order than with the XCD-aware one.
    // kslab 0: planes per work item from the number of active blocks
    // (auto_kslab)
    int kslab = 0;
    int xcd = 0;
    int kslab_last = 0;
    int xcd_last = 0;
    // 16 planes per work item from 512 active blocks on (a whole round of the
    // GPU's workgroup slots), 8 from 256, else 4: on a 64-block box 4-plane
    // slabs make the step 2.4x faster, at 512 and more blocks 16 planes are
    // within 1% of the fastest shape
    int auto_kslab() const { return nlist_ >= 512 ? 16 : (nlist_ >= 256 ? 8 : 4); }
    int stage_kslab(bool last_kind) const {
        const int k = last_kind ? kslab_last : kslab;
        return k ? k : auto_kslab();
    }
    // host time (ms) of table rebuilds and graph captures / instantiations,
    // and the number of graphs built, since construction
    double build_ms = 0.0;
    int64_t graph_builds = 0;

private:
    int rebuild(std::string &err);
    int enqueue_fill(int buf, std::string &err, bool restricted = false);
    int enqueue_correct(int out, double bw, bool last, bool fill, std::string &err);
    int enqueue_stage(int kind, int in, int out, double bw, bool fill, std::string &err);
    int enqueue_step(bool cfl_dt, std::string &err);
    int tbegin(int kind, std::string &err);
    int tend(int kind, std::string &err);
    int tcollect(std::string &err);
    void free_all();

    EngineConfig cfg_{};
    bool owns_ = true;            // false: the arrays live in the caller's pool
    int nvar_ = 5;
    std::vector<MeshSlot> slots_;
    RangeAlloc blocks_, halos_, fregs_;
    // pool
    double *U_[3] = {nullptr, nullptr, nullptr}, *XE_[3] = {nullptr, nullptr, nullptr};   // [2]: SSP-RK3 only
    double *halo_ = nullptr, *freg_ = nullptr;
    BlockDesc *desc_ = nullptr;
    MeshParams *mp_ = nullptr;
    unsigned long long *smax_ = nullptr;
    unsigned long long *cmax_ = nullptr;   // MHD: second half of the smax_ allocation
    // concatenated tables of the active meshes
    int *d_list_ = nullptr, *d_meshes_ = nullptr, *d_perm_ = nullptr;
    RestrictTask *d_restrict_ = nullptr;
    ProlongTask *d_prolong_ = nullptr;
    RefluxTask *d_reflux_ = nullptr;
    int nlist_ = 0, nmeshes_ = 0, nrestrict_ = 0, nreflux_ = 0;
    bool rr_indep_ = false;   // flux correction and restriction touch different blocks
    bool ghosts_valid_ = false;   // halo slabs hold the ghost fill of U[0] (Euler)
    std::vector<int> pro_off_, pro_cnt_;
    std::vector<char> pro_dep_;   // [level] waits for the level below (some mesh)
    bool dirty_ = true;
    // graph of one CFL step
    hipGraph_t graph_ = nullptr;
    hipGraphExec_t graph_exec_ = nullptr;
    bool capturing_ = false;
    // timing
    int timing_ = 0;              // bit mask of timed kernel classes
    std::vector<hipEvent_t> events_;
    std::vector<int> event_kind_;
    size_t pairs_used_ = 0;
    double ms_[4] = {0, 0, 0, 0};
    int64_t launches_[4] = {0, 0, 0, 0};
};


} // namespace agile
