// engine.cpp -- device block pool, table rebuild, step sequencing (eager or
// one captured hipGraph per step), autotuning of the stage kernel's shape and
// kernel timing.  See engine.hpp.
#include "engine.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

namespace agile {

#define CHK(call)                                                                         \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) {                                                           \
            err = std::string(#call) + ": " + hipGetErrorString(e_);                      \
            return AGILE_EDEVICE;                                                         \
        }                                                                                 \
    } while (0)

// ---------------------------------------------------------------------------
// RangeAlloc

void RangeAlloc::reset(int cap) {
    free_.clear();
    if (cap > 0) free_[0] = cap;
    free_total_ = std::max(cap, 0);
}

int RangeAlloc::alloc(int n) {
    if (n <= 0) return 0;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second >= n) {
            const int start = it->first, len = it->second;
            free_.erase(it);
            if (len > n) free_[start + n] = len - n;
            free_total_ -= n;
            return start;
        }
    }
    return -1;
}

void RangeAlloc::release(int start, int n) {
    if (n <= 0) return;
    auto it = free_.emplace(start, n).first;
    free_total_ += n;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        free_.erase(nx);
    }
    if (it != free_.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            free_.erase(it);
        }
    }
}

bool RangeAlloc::can_alloc(int n) const {
    if (n <= 0) return true;
    for (const auto &kv : free_)
        if (kv.second >= n) return true;
    return false;
}

// ---------------------------------------------------------------------------
// host copies between blocks of (16 te)^3 cells and 16^3 tiles (caller tile q
// = sub-tile q mod te^3 of block q / te^3, x fastest; tiles in device order
// perm[q] of the local range)

static void tile_copy(double *blocks, double *tiles, const int *perm, int ntiles, int nv, int te, bool to_tiles) {
    const int t3 = te * te * te, B = BN * te;
    for (int q = 0; q < ntiles; ++q) {
        const int bq = q / t3, t = q - bq * t3;
        const int tx = t % te, ty = (t / te) % te, tz = t / (te * te);
        double *tile = tiles + size_t(perm[q]) * nv * CELLS;
        for (int v = 0; v < nv; ++v)
            for (int k = 0; k < BN; ++k)
                for (int j = 0; j < BN; ++j) {
                    double *row = blocks + ((size_t(bq) * nv + v) * B + (tz * BN + k)) * B * B +
                                  size_t(ty * BN + j) * B + tx * BN;
                    double *trow = tile + size_t(v) * CELLS + (k * BN + j) * BN;
                    if (to_tiles) std::memcpy(trow, row, BN * sizeof(double));
                    else std::memcpy(row, trow, BN * sizeof(double));
                }
    }
}

void tiles_from_blocks(const double *blocks, double *tiles, const int *perm, int ntiles, int nv, int te) {
    tile_copy(const_cast<double *>(blocks), tiles, perm, ntiles, nv, te, true);
}

void blocks_from_tiles(const double *tiles, double *blocks, const int *perm, int ntiles, int nv, int te) {
    tile_copy(blocks, const_cast<double *>(tiles), perm, ntiles, nv, te, false);
}

// ---------------------------------------------------------------------------
// Engine

Engine::~Engine() { free_all(); }

void Engine::free_all() {
    if (graph_exec_) (void)hipGraphExecDestroy(graph_exec_);
    if (graph_) (void)hipGraphDestroy(graph_);
    graph_exec_ = nullptr;
    graph_ = nullptr;
    for (MeshSlot &s : slots_) s.d_perm = nullptr;
    void *ptrs[] = {U_[0], U_[1], U_[2], XE_[0], XE_[1], XE_[2], halo_, freg_, desc_, mp_, smax_,
                    d_list_, d_meshes_, d_restrict_, d_prolong_, d_reflux_, d_perm_};
    if (owns_)   // arrays carved from a caller's pool are the caller's
        for (void *p : ptrs)
            if (p) (void)hipFree(p);
    U_[0] = U_[1] = U_[2] = XE_[0] = XE_[1] = XE_[2] = halo_ = freg_ = nullptr;
    cmax_ = nullptr;
    desc_ = nullptr;
    mp_ = nullptr;
    smax_ = nullptr;
    d_list_ = d_meshes_ = d_perm_ = nullptr;
    d_restrict_ = nullptr;
    d_prolong_ = nullptr;
    d_reflux_ = nullptr;
    for (hipEvent_t e : events_) (void)hipEventDestroy(e);
    events_.clear();
    event_kind_.clear();
    pairs_used_ = 0;
}

// Device arrays of an engine, in the order they are carved from a pool.
enum {
    A_U0, A_U1, A_X0, A_X1, A_U2, A_X2, A_HALO, A_FREG, A_DESC, A_MP, A_SMAX, A_LIST, A_PERM, A_MESHES,
    A_RESTRICT, A_PROLONG, A_REFLUX, A_COUNT
};

// Bytes of each array for config c (0: not used).
static void array_bytes(const EngineConfig &c, size_t out[A_COUNT]) {
    const int nv = c.physics == AGILE_MHD_GLM ? 9 : 5;
    const bool rk3 = c.rk == 3;
    const size_t nb = size_t(c.cap_blocks), nh = size_t(std::max(c.cap_halo, 1)),
                 nf = size_t(std::max(c.cap_freg, 1)), nm = size_t(c.cap_meshes);
    const size_t state = nb * nv * CELLS * sizeof(double), xe = nb * nv * XE_CELLS * sizeof(double);
    out[A_U0] = state;
    out[A_U1] = state;
    out[A_X0] = xe;
    out[A_X1] = xe;
    out[A_U2] = rk3 ? state : 0;
    out[A_X2] = rk3 ? xe : 0;
    out[A_HALO] = nh * nv * SLAB * sizeof(double);
    out[A_FREG] = nf * nv * REG * sizeof(double);
    out[A_DESC] = nb * sizeof(BlockDesc);
    out[A_MP] = nm * sizeof(MeshParams);
    out[A_SMAX] = 2 * nb * sizeof(unsigned long long);   // signal rate, then MHD speed
    out[A_LIST] = nb * sizeof(int);
    out[A_PERM] = nb * sizeof(int);
    out[A_MESHES] = 2 * nm * sizeof(int);
    out[A_RESTRICT] = nh * sizeof(RestrictTask);
    out[A_PROLONG] = nh * sizeof(ProlongTask);
    out[A_REFLUX] = nb * sizeof(RefluxTask);
}

constexpr size_t POOL_ALIGN = 256;   // every carved array starts on a 256-byte boundary

size_t engine_device_bytes(const EngineConfig &c) {
    size_t b[A_COUNT], total = 0;
    array_bytes(c, b);
    for (size_t x : b) total += (x + POOL_ALIGN - 1) / POOL_ALIGN * POOL_ALIGN;
    return total;
}

int Engine::init(const EngineConfig &c, std::string &err) {
    if (c.physics != AGILE_EULER && c.physics != AGILE_MHD_GLM && c.physics != AGILE_SRHD) {
        err = "unknown physics";
        return AGILE_EINVAL;
    }
    if (c.physics == AGILE_SRHD && c.riemann != AGILE_LF) {
        err = "the SRHD module takes the LF flux";
        return AGILE_EINVAL;
    }
    if ((c.limiter != 0 && c.limiter != 1) || (c.rk != 2 && c.rk != 3) ||
        (c.physics == AGILE_MHD_GLM && (c.limiter != 0 || c.rk != 2 || c.riemann != AGILE_HLL))) {
        err = "unsupported scheme (MHD: HLL, minmod, SSP-RK2)";
        return AGILE_EINVAL;
    }
    if (c.cap_blocks < 1 || c.cap_meshes < 1 || c.cap_halo < 0 || c.cap_freg < 0) {
        err = "bad pool capacity";
        return AGILE_EINVAL;
    }
    if (c.pool && (reinterpret_cast<uintptr_t>(c.pool) % POOL_ALIGN) != 0) {
        err = "caller device pool must be 256-byte aligned";
        return AGILE_EINVAL;
    }
    cfg_ = c;
    nvar_ = c.physics == AGILE_MHD_GLM ? 9 : 5;
    const bool mhd = nvar_ == 9;
    slots_.assign(size_t(c.cap_meshes), MeshSlot{});
    blocks_.reset(c.cap_blocks);
    halos_.reset(c.cap_halo);
    fregs_.reset(c.cap_freg);
    const size_t nm = size_t(c.cap_meshes);
    void **dst[A_COUNT] = {
        (void **)&U_[0], (void **)&U_[1], (void **)&XE_[0], (void **)&XE_[1],
        (void **)&U_[2], (void **)&XE_[2], (void **)&halo_, (void **)&freg_, (void **)&desc_, (void **)&mp_,
        (void **)&smax_, (void **)&d_list_, (void **)&d_perm_, (void **)&d_meshes_, (void **)&d_restrict_,
        (void **)&d_prolong_, (void **)&d_reflux_};
    size_t bytes[A_COUNT];
    array_bytes(c, bytes);
    if (c.pool) {
        // carve every array from the caller's memory; nothing is allocated
        const size_t need = engine_device_bytes(c);
        if (need > c.pool_bytes) {
            err = "caller device pool too small: " + std::to_string(c.pool_bytes) + " bytes given, " +
                  std::to_string(need) + " needed";
            return AGILE_ENOMEM;
        }
        owns_ = false;
        char *at = static_cast<char *>(c.pool);
        for (int a = 0; a < A_COUNT; ++a) {
            *dst[a] = bytes[a] ? at : nullptr;
            at += (bytes[a] + POOL_ALIGN - 1) / POOL_ALIGN * POOL_ALIGN;
        }
    } else {
        owns_ = true;
        for (int a = 0; a < A_COUNT; ++a) {
            *dst[a] = nullptr;
            if (bytes[a] == 0) continue;
            if (hipMalloc(dst[a], bytes[a]) != hipSuccess) {
                (void)hipGetLastError();
                *dst[a] = nullptr;
                free_all();
                err = "device pool allocation of " + std::to_string(bytes[a]) + " bytes failed";
                return AGILE_ENOMEM;
            }
        }
    }
    cmax_ = mhd ? smax_ + c.cap_blocks : nullptr;
    // second half of d_meshes_: the identity map slot -> slot, for single-mesh reductions
    std::vector<int> ident(nm);
    for (size_t q = 0; q < nm; ++q) ident[q] = int(q);
    CHK(hipMemcpy(d_meshes_ + nm, ident.data(), nm * sizeof(int), hipMemcpyHostToDevice));
    pro_off_.assign(MAXLEV + 1, 0);
    pro_cnt_.assign(MAXLEV + 1, 0);
    pro_dep_.assign(MAXLEV + 1, 0);
    dirty_ = true;
    return AGILE_OK;
}

int Engine::plan(const agile_config &cfg, int64_t n, const agile_block_desc *b, Plan &P, std::string &err) const {
    if (cfg.physics != cfg_.physics || cfg.riemann != cfg_.riemann || cfg.precision != cfg_.precision) {
        err = "mesh physics / solver / precision differ from the engine's";
        return AGILE_EINVAL;
    }
    PlanInput in{{cfg.base_blocks[0], cfg.base_blocks[1], cfg.base_blocks[2]}, cfg.max_level};
    if (build_plan(in, n, b, P) != AGILE_OK) {
        err = P.error;
        return AGILE_EINVAL;
    }
    return AGILE_OK;
}

bool Engine::fits(const Plan &P) const {
    bool slot = false;
    for (const MeshSlot &s : slots_)
        if (!s.used) slot = true;
    return slot && blocks_.can_alloc(int(P.n)) && halos_.can_alloc(P.nhalo) && fregs_.can_alloc(P.nfreg);
}

bool Engine::fits_replacing(int s, const Plan &P) const {
    if (s < 0 || s >= int(slots_.size()) || !slots_[s].used) return fits(P);
    const MeshSlot &S = slots_[s];
    RangeAlloc b = blocks_, h = halos_, f = fregs_;
    b.release(S.first, int(S.plan.n));
    h.release(S.halo0, S.plan.nhalo);
    f.release(S.freg0, S.plan.nfreg);
    return b.can_alloc(int(P.n)) && h.can_alloc(P.nhalo) && f.can_alloc(P.nfreg);
}

int Engine::add(const agile_config &cfg, Plan &&P, const double *u, int u_on_device, int64_t steps, uint64_t tag,
                int *slot_out, std::string &err, const MeshParams *carry, int u_edge, int slot_edge) {
    if (u_edge < 1 || slot_edge < 1 || P.n % (int64_t(u_edge) * u_edge * u_edge) != 0) {
        err = "tile layout does not match the plan";
        return AGILE_EINVAL;
    }
    int s = -1;
    for (int q = 0; q < int(slots_.size()); ++q)
        if (!slots_[q].used) {
            s = q;
            break;
        }
    const int n = int(P.n);
    if (s < 0 || !fits(P)) {
        err = "no room in the device pool";
        return AGILE_ENOMEM;
    }
    const int first = blocks_.alloc(n), halo0 = halos_.alloc(P.nhalo), freg0 = fregs_.alloc(P.nfreg);
    // rewrite the plan to pool indices
    for (BlockDesc &D : P.desc) {
        for (int f = 0; f < 6; ++f) {
            D.nb[f] = D.nb[f] >= 0 ? D.nb[f] + first : -((-D.nb[f] - 1) + halo0 + 1);
            if (D.freg[f] >= 0) D.freg[f] += freg0;
        }
        D.mesh = s;
    }
    for (RestrictTask &t : P.restrict_tasks) {
        t.slot += halo0;
        t.block += first;
        for (int q = 0; q < 4; ++q) t.fine[q] += first;
    }
    for (auto &lv : P.prolong)
        for (ProlongTask &t : lv) {
            t.slot += halo0;
            t.block += first;
            t.coarse += first;
        }
    for (RefluxTask &r : P.reflux) {
        r.block += first;
        r.mesh = s;
        for (int f = 0; f < r.nface; ++f) {
            r.cslot[f] += freg0;
            for (int q = 0; q < 4; ++q) r.fslot[f][q] += freg0;
        }
    }
    MeshSlot &S = slots_[s];
    S = MeshSlot{};
    S.used = true;
    S.active = true;
    S.cfg = cfg;
    S.first = first;
    S.halo0 = halo0;
    S.freg0 = freg0;
    S.steps_target = steps;
    S.steps_done = 0;
    S.tag = tag;
    S.tile_edge = slot_edge;
    const hipStream_t st = cfg_.stream;
    MeshParams hp{};
    hp.gamma = cfg.gamma;
    hp.cfl = cfg.cfl;
    hp.physics = cfg.physics;
    hp.inv_dx1 = (double(cfg.base_blocks[0]) * BN) / (cfg.hi[0] - cfg.lo[0]);
    hp.glm_alpha = cfg.glm_alpha;
    hp.first_block = first;
    hp.nblocks = n;
    if (carry) {
        hp.t = carry->t;
        hp.dt = carry->dt;
        hp.flags = carry->flags;
    }
    auto undo = [&]() {
        blocks_.release(first, n);
        halos_.release(halo0, P.nhalo);
        fregs_.release(freg0, P.nfreg);
        S = MeshSlot{};
    };
    S.d_perm = d_perm_ + first;   // the mesh's block range of the pool-wide permutation
    const size_t per = size_t(nvar_) * CELLS;
    hipError_t e = hipSuccess;
    e = e ? e : hipMemcpyAsync(desc_ + first, P.desc.data(), size_t(n) * sizeof(BlockDesc), hipMemcpyHostToDevice, st);
    e = e ? e : hipMemcpyAsync(mp_ + s, &hp, sizeof(MeshParams), hipMemcpyHostToDevice, st);
    e = e ? e : hipMemcpyAsync(S.d_perm, P.perm.data(), size_t(n) * sizeof(int), hipMemcpyHostToDevice, st);
    std::vector<double> tmp;
    if (!e) {
        if (u_on_device) {
            e = u_edge == 1 ? launch_permute(u, U_[0], S.d_perm, first, n, int(per), 0, st)
                            : launch_permute_tiles(u, U_[0], S.d_perm, first, n, nvar_, u_edge, 0, st);
        } else {
            tmp.resize(size_t(n) * per);
            if (u_edge == 1) {
                for (int q = 0; q < n; ++q)
                    std::memcpy(&tmp[size_t(P.perm[q]) * per], u + size_t(q) * per, per * sizeof(double));
            } else {
                tiles_from_blocks(u, tmp.data(), P.perm.data(), n, nvar_, u_edge);
            }
            e = hipMemcpyAsync(U_[0] + size_t(first) * per, tmp.data(), tmp.size() * sizeof(double),
                               hipMemcpyHostToDevice, st);
        }
    }
    if (XE_[0]) e = e ? e : launch_xexport(U_[0], XE_[0], first, n, nvar_, st);
    e = e ? e : launch_smax(desc_, mp_, U_[0], smax_, cmax_, first, n, nvar_, st);
    e = e ? e : launch_mesh_reduce(mp_, d_meshes_ + cfg_.cap_meshes + s, 1, smax_, cmax_, 2, st);
    e = e ? e : hipStreamSynchronize(st);
    if (e) {
        undo();
        err = std::string("mesh upload: ") + hipGetErrorString(e);
        return AGILE_EDEVICE;
    }
    S.plan = std::move(P);
    dirty_ = true;
    *slot_out = s;
    return AGILE_OK;
}

int Engine::remove(int s) {
    if (s < 0 || s >= int(slots_.size()) || !slots_[s].used) return AGILE_EINVAL;
    (void)hipStreamSynchronize(cfg_.stream);
    MeshSlot &S = slots_[s];
    blocks_.release(S.first, int(S.plan.n));
    halos_.release(S.halo0, S.plan.nhalo);
    fregs_.release(S.freg0, S.plan.nfreg);
    S = MeshSlot{};
    dirty_ = true;
    return AGILE_OK;
}

int Engine::set_progress(int s, int64_t steps_done) {
    if (s < 0 || s >= int(slots_.size()) || !slots_[s].used || steps_done < 0) return AGILE_EINVAL;
    slots_[s].steps_done = steps_done;
    return AGILE_OK;
}

int Engine::set_active(int s, bool a) {
    if (s < 0 || s >= int(slots_.size()) || !slots_[s].used) return AGILE_EINVAL;
    if (slots_[s].active != a) {
        slots_[s].active = a;
        dirty_ = true;
    }
    return AGILE_OK;
}

int Engine::rebuild(std::string &err) {
    if (!dirty_) return AGILE_OK;
    const auto t0 = std::chrono::steady_clock::now();
    struct Clock {
        double &ms;
        std::chrono::steady_clock::time_point t0;
        ~Clock() { ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count(); }
    } clock{build_ms, t0};
    std::vector<int> list, meshes;
    std::vector<RestrictTask> res;
    std::vector<ProlongTask> pro;
    std::vector<RefluxTask> ref;
    for (int s = 0; s < int(slots_.size()); ++s) {
        const MeshSlot &S = slots_[s];
        if (!S.used || !S.active) continue;
        meshes.push_back(s);
        for (int q = 0; q < int(S.plan.n); ++q) list.push_back(S.first + q);
        res.insert(res.end(), S.plan.restrict_tasks.begin(), S.plan.restrict_tasks.end());
        ref.insert(ref.end(), S.plan.reflux.begin(), S.plan.reflux.end());
    }
    for (int l = 0; l <= MAXLEV; ++l) {
        pro_off_[l] = int(pro.size());
        pro_dep_[l] = 0;
        for (int s = 0; s < int(slots_.size()); ++s) {
            const MeshSlot &S = slots_[s];
            if (!S.used || !S.active || l >= int(S.plan.prolong.size())) continue;
            pro.insert(pro.end(), S.plan.prolong[l].begin(), S.plan.prolong[l].end());
            pro_dep_[l] |= S.plan.prolong_dep[l];
        }
        pro_cnt_[l] = int(pro.size()) - pro_off_[l];
    }
    const hipStream_t st = cfg_.stream;
    if (!list.empty()) CHK(hipMemcpyAsync(d_list_, list.data(), list.size() * sizeof(int), hipMemcpyHostToDevice, st));
    if (!meshes.empty())
        CHK(hipMemcpyAsync(d_meshes_, meshes.data(), meshes.size() * sizeof(int), hipMemcpyHostToDevice, st));
    if (!res.empty())
        CHK(hipMemcpyAsync(d_restrict_, res.data(), res.size() * sizeof(RestrictTask), hipMemcpyHostToDevice, st));
    if (!pro.empty())
        CHK(hipMemcpyAsync(d_prolong_, pro.data(), pro.size() * sizeof(ProlongTask), hipMemcpyHostToDevice, st));
    if (!ref.empty())
        CHK(hipMemcpyAsync(d_reflux_, ref.data(), ref.size() * sizeof(RefluxTask), hipMemcpyHostToDevice, st));
    CHK(hipStreamSynchronize(st));
    nlist_ = int(list.size());
    nmeshes_ = int(meshes.size());
    nrestrict_ = int(res.size());
    nreflux_ = int(ref.size());
    // the flux correction and the restriction may share a launch when no
    // corrected block is read by a restriction task
    {
        std::vector<char> corrected(size_t(cfg_.cap_blocks), 0);
        for (const RefluxTask &r : ref) corrected[r.block] = 1;
        rr_indep_ = true;
        for (const RestrictTask &t : res)
            for (int q = 0; q < 4; ++q) rr_indep_ = rr_indep_ && !corrected[t.fine[q]];
    }
    if (graph_exec_) (void)hipGraphExecDestroy(graph_exec_);
    if (graph_) (void)hipGraphDestroy(graph_);
    graph_exec_ = nullptr;
    graph_ = nullptr;
    dirty_ = false;
    ghosts_valid_ = false;   // meshes were added, removed or (de)activated
    return AGILE_OK;
}

// ---------------------------------------------------------------------------
// timing

int Engine::tbegin(int kind, std::string &err) {
    if (!((timing_ >> kind) & 1) || capturing_) return AGILE_OK;
    if (pairs_used_ == event_kind_.size()) {
        hipEvent_t a, b;
        CHK(hipEventCreate(&a));
        CHK(hipEventCreate(&b));
        events_.push_back(a);
        events_.push_back(b);
        event_kind_.push_back(kind);
    }
    event_kind_[pairs_used_] = kind;
    CHK(hipEventRecord(events_[2 * pairs_used_], cfg_.stream));
    return AGILE_OK;
}

int Engine::tend(int kind, std::string &err) {
    if (!((timing_ >> kind) & 1) || capturing_) return AGILE_OK;
    CHK(hipEventRecord(events_[2 * pairs_used_ + 1], cfg_.stream));
    pairs_used_++;
    return AGILE_OK;
}

int Engine::tcollect(std::string &err) {
    if (pairs_used_ == 0) return AGILE_OK;
    CHK(hipStreamSynchronize(cfg_.stream));
    for (size_t q = 0; q < pairs_used_; ++q) {
        float t = 0.f;
        CHK(hipEventElapsedTime(&t, events_[2 * q], events_[2 * q + 1]));
        ms_[event_kind_[q]] += t;
        launches_[event_kind_[q]] += 1;
    }
    pairs_used_ = 0;
    return AGILE_OK;
}

int Engine::profile(int kinds, std::string &err) {
    if (kinds & 16) {   // keep: switch the timed classes only (no wait, totals kept)
        timing_ = kinds & 15;
        return AGILE_OK;
    }
    int e = tcollect(err);
    if (e) return e;
    timing_ = kinds & 15;
    for (int k = 0; k < 4; ++k) {
        ms_[k] = 0.0;
        launches_[k] = 0;
    }
    return AGILE_OK;
}

int Engine::profile_read(int kind, double &ms, int64_t &launches, std::string &err) {
    if (kind < 0 || kind > 3) return AGILE_EINVAL;
    int e = tcollect(err);
    if (e) return e;
    ms = ms_[kind];
    launches = launches_[kind];
    return AGILE_OK;
}

#define TIMED(kind, call)                   \
    do {                                    \
        int te_ = tbegin(kind, err);        \
        if (te_) return te_;                \
        CHK(call);                          \
        if ((te_ = tend(kind, err))) return te_; \
    } while (0)

// ---------------------------------------------------------------------------
// step sequencing

int Engine::enqueue_fill(int buf, std::string &err, bool restricted) {
    const hipStream_t st = cfg_.stream;
    if (nrestrict_ > 0 && !restricted)
        TIMED(AGILE_K_FILL, launch_restrict(d_restrict_, nrestrict_, U_[buf], halo_, nvar_, st));
    // levels are launched together until one depends on the level below
    const int srhd = cfg_.physics == AGILE_SRHD;   // SRHD prolongs primitives
    int first = 0, count = 0;
    for (int l = 0; l <= MAXLEV; ++l) {
        if (pro_cnt_[l] == 0) continue;
        if (pro_dep_[l] && count > 0) {
            TIMED(AGILE_K_FILL, launch_prolong(d_prolong_ + first, count, desc_, mp_, U_[buf], XE_[buf], halo_, nvar_, srhd, st));
            count = 0;
        }
        if (count == 0) first = pro_off_[l];
        count += pro_cnt_[l];
    }
    if (count > 0)
        TIMED(AGILE_K_FILL, launch_prolong(d_prolong_ + first, count, desc_, mp_, U_[buf], XE_[buf], halo_, nvar_, srhd, st));
    return AGILE_OK;
}

// Flux correction of stage output `out` with the stage's weight bw of dt L;
// with fill set, followed by the ghost fill of `out` -- its restriction in the
// same launch as the correction when the two touch different blocks.
int Engine::enqueue_correct(int out, double bw, bool last, bool fill, std::string &err) {
    const hipStream_t st = cfg_.stream;
    double *xe = XE_[out];
    unsigned long long *cm = nvar_ == 9 ? cmax_ : nullptr;
    bool restricted = false;
    if (nreflux_ > 0) {
        if (fill && nrestrict_ > 0 && rr_indep_) {
            TIMED(AGILE_K_REFLUX, launch_reflux_restrict(d_reflux_, nreflux_, d_restrict_, nrestrict_, mp_, U_[out], xe,
                                                         freg_, halo_, smax_, cm, nvar_, bw, last, st));
            restricted = true;
        } else {
            TIMED(AGILE_K_REFLUX, launch_reflux(d_reflux_, nreflux_, mp_, U_[out], xe, freg_, smax_, cm, nvar_, bw, last, st));
        }
    }
    return fill ? enqueue_fill(out, err, restricted) : AGILE_OK;
}

// One stage: kind (1 first, 2 last SSP-RK2, 3 middle / 4 last SSP-RK3) from
// buffer `in` into buffer `out`, U^n in buffer 0; then the flux correction of
// the output and, with fill set, the ghost fill of the output.
int Engine::enqueue_stage(int kind, int in, int out, double bw, bool fill, std::string &err) {
    const hipStream_t st = cfg_.stream;
    const bool last = kind == 2 || kind == 4;
    if (nvar_ == 9) {
        SweepArgs m{};
        m.desc = desc_;
        m.mp = mp_;
        m.Uin = U_[in];
        m.Uout = U_[out];
        m.Un = kind == 1 ? nullptr : U_[0];
        m.XEin = XE_[in];
        m.XEout = XE_[out];
        m.halo = halo_;
        m.freg = freg_;
        m.smax = smax_;
        m.cmax = cmax_;
        m.list = d_list_;
        m.nblocks = nlist_;
        TIMED(AGILE_K_STAGE, launch_mhd_stage(m, kind, cfg_.precision, st));
        return enqueue_correct(out, bw, last, fill, err);
    }
    StageArgs a{};
    a.desc = desc_;
    a.mp = mp_;
    a.halo = halo_;
    a.freg = freg_;
    a.smax = smax_;
    a.list = d_list_;
    a.nblocks = nlist_;
    const bool last_kind = kind == 2 || kind == 4;
    a.kslab = stage_kslab(last_kind);
    a.xcd = last_kind ? xcd_last : xcd;
    a.stage = kind;
    a.limiter = cfg_.limiter;
    a.Uin = U_[in];
    a.Uout = U_[out];
    a.Un = kind == 1 ? nullptr : U_[0];
    a.XEin = XE_[in];
    a.XEout = XE_[out];
    TIMED(AGILE_K_STAGE, launch_stage(a, stage_solver(), cfg_.precision, st));
    return enqueue_correct(out, bw, last, fill, err);
}

int Engine::enqueue_step(bool cfl_dt, std::string &err) {
    const hipStream_t st = cfg_.stream;
    int e;
    const bool mhd = nvar_ == 9;
    // CFL step: dt (and the GLM speed c_h) from the state's reductions; given
    // dt: c_h only
    if (cfl_dt || mhd) TIMED(AGILE_K_DT, launch_mesh_reduce(mp_, d_meshes_, nmeshes_, smax_, cmax_, cfl_dt ? 1 : 3, st));
    if (mhd) TIMED(AGILE_K_DT, launch_glm_decay(desc_, mp_, U_[0], XE_[0], d_list_, nlist_, 0.5, st));
    // Euler steps end with the ghost fill of their result (its restriction
    // shares the last flux correction's launch), so a step starts with valid
    // ghosts unless the set of meshes changed; MHD fills after the psi decay
    if (mhd || !ghosts_valid_)
        if ((e = enqueue_fill(0, err))) return e;
    if ((e = enqueue_stage(1, 0, 1, 1.0, true, err))) return e;
    if (cfg_.rk == 3) {
        if ((e = enqueue_stage(3, 1, 2, 0.25, true, err))) return e;
        if ((e = enqueue_stage(4, 2, 0, 2.0 / 3.0, !mhd, err))) return e;
    } else {
        if ((e = enqueue_stage(2, 1, 0, 0.5, !mhd, err))) return e;
    }
    // MHD: the second half of the psi decay is applied by the last stage and
    // its flux correction (k_mhd_stage<2>, k_reflux)
    TIMED(AGILE_K_DT, launch_mesh_reduce(mp_, d_meshes_, nmeshes_, smax_, cmax_, 0, st));
    ghosts_valid_ = !mhd;
    return AGILE_OK;
}

int Engine::step_cfl(int nsteps, std::string &err) {
    int e = rebuild(err);
    if (e) return e;
    if (nlist_ == 0) return AGILE_OK;
    const hipStream_t st = cfg_.stream;
    for (int q = 0; q < nsteps; ++q) {
        if (use_graph && !timing_ && st != nullptr) {
            // the captured step assumes valid ghosts at its start (Euler)
            if (!ghosts_valid_ && nvar_ != 9) {
                if ((e = enqueue_fill(0, err))) return e;
                ghosts_valid_ = true;
            }
            if (!graph_exec_) {
                struct Clock {
                    double &ms;
                    std::chrono::steady_clock::time_point t0;
                    ~Clock() {
                        ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
                    }
                } clock{build_ms, std::chrono::steady_clock::now()};
                graph_builds++;
                CHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                capturing_ = true;
                std::string e2;
                const int rc = enqueue_step(true, e2);
                capturing_ = false;
                hipGraph_t g = nullptr;
                const hipError_t ec = hipStreamEndCapture(st, &g);
                if (rc || ec != hipSuccess) {
                    if (g) (void)hipGraphDestroy(g);
                    err = rc ? e2 : std::string("graph capture: ") + hipGetErrorString(ec);
                    return rc ? rc : AGILE_EDEVICE;
                }
                graph_ = g;
                CHK(hipGraphInstantiate(&graph_exec_, graph_, nullptr, nullptr, 0));
            }
            CHK(hipGraphLaunch(graph_exec_, st));
        } else {
            if ((e = enqueue_step(true, err))) return e;
        }
        for (MeshSlot &S : slots_)
            if (S.used && S.active) S.steps_done++;
        if (pairs_used_ > 4096 && (e = tcollect(err))) return e;
    }
    return AGILE_OK;
}

int Engine::step_dt(int s, double dt, std::string &err) {
    int e = rebuild(err);
    if (e) return e;
    if (nmeshes_ != 1 || !slots_[s].active) {
        err = "a step with a given dt needs exactly one active mesh";
        return AGILE_ESTATE;
    }
    CHK(launch_set_dt(mp_, s, dt, cfg_.stream));
    if ((e = enqueue_step(false, err))) return e;
    slots_[s].steps_done++;
    if (pairs_used_ > 4096) return tcollect(err);
    return AGILE_OK;
}

int Engine::fill_ghosts(std::string &err) {
    int e = rebuild(err);
    if (e) return e;
    if ((e = enqueue_fill(0, err))) return e;
    ghosts_valid_ = nvar_ != 9;
    return AGILE_OK;
}

int Engine::read_params(int s, MeshParams &hp, std::string &err) {
    CHK(hipMemcpyAsync(&hp, mp_ + s, sizeof(MeshParams), hipMemcpyDeviceToHost, cfg_.stream));
    CHK(hipStreamSynchronize(cfg_.stream));
    return AGILE_OK;
}

int Engine::read_state(int s, double *out, int out_on_device, std::string &err) {
    const MeshSlot &S = slots_[s];
    const int n = int(S.plan.n);
    const size_t per = size_t(nvar_) * CELLS;
    const hipStream_t st = cfg_.stream;
    if (out_on_device) {
        if (S.tile_edge == 1) CHK(launch_permute(U_[0], out, S.d_perm, S.first, n, int(per), 1, st));
        else CHK(launch_permute_tiles(U_[0], out, S.d_perm, S.first, n, nvar_, S.tile_edge, 1, st));
        return AGILE_OK;
    }
    std::vector<double> tmp(size_t(n) * per);
    CHK(hipMemcpyAsync(tmp.data(), U_[0] + size_t(S.first) * per, tmp.size() * sizeof(double), hipMemcpyDeviceToHost,
                       st));
    CHK(hipStreamSynchronize(st));
    if (S.tile_edge == 1) {
        for (int q = 0; q < n; ++q)
            std::memcpy(out + size_t(q) * per, &tmp[size_t(S.plan.perm[q]) * per], per * sizeof(double));
    } else {
        blocks_from_tiles(tmp.data(), out, S.plan.perm.data(), n, nvar_, S.tile_edge);
    }
    return AGILE_OK;
}

int Engine::lohner(int s, int v, double eps, double *out_host, std::string &err) {
    if (s < 0 || s >= int(slots_.size()) || !slots_[s].used) return AGILE_EINVAL;
    if (v < 0 || v >= nvar_ || !(eps > 0.0)) {
        err = "estimator: variable out of range or eps not positive";
        return AGILE_EINVAL;
    }
    const MeshSlot &S = slots_[s];
    const int n = int(S.plan.n);
    const hipStream_t st = cfg_.stream;
    int e = fill_ghosts(err);
    if (e) return e;
    // U[1] is free between steps: the per-block maxima go to its mesh range
    double *d = U_[1] + size_t(S.first) * nvar_ * CELLS;
    CHK(launch_lohner(desc_, U_[0], halo_, S.first, n, nvar_, v, eps, d, st));
    std::vector<double> tmp(static_cast<size_t>(n));
    CHK(hipMemcpyAsync(tmp.data(), d, tmp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    CHK(hipStreamSynchronize(st));
    for (int q = 0; q < n; ++q) out_host[q] = tmp[size_t(S.plan.perm[q])];
    return AGILE_OK;
}

int Engine::remap(int s, const std::vector<RegridSource> &src, double *out_dev, std::string &err,
                  RemapTask *d_tasks) {
    if (s < 0 || s >= int(slots_.size()) || !slots_[s].used) return AGILE_EINVAL;
    const MeshSlot &S = slots_[s];
    const int n = int(S.plan.n);
    std::vector<RemapTask> t(src.size());
    for (size_t i = 0; i < src.size(); ++i) {
        t[i].kind = src[i].kind;
        t[i].octant = src[i].octant;
        const int m = src[i].kind == 2 ? 8 : 1;
        for (int o = 0; o < 8; ++o) {
            const int c = o < m ? src[i].src[o] : -1;
            if (o < m && (c < 0 || c >= n)) {
                err = "remap: source block out of range";
                return AGILE_EINVAL;
            }
            t[i].src[o] = c >= 0 ? S.first + S.plan.perm[c] : -1;
        }
    }
    int e = fill_ghosts(err);
    if (e) return e;
    const hipStream_t st = cfg_.stream;
    RemapTask *d_t = d_tasks;
    if (!d_t) CHK(hipMalloc(&d_t, std::max<size_t>(1, t.size()) * sizeof(RemapTask)));
    hipError_t he = hipMemcpyAsync(d_t, t.data(), t.size() * sizeof(RemapTask), hipMemcpyHostToDevice, st);
    if (he == hipSuccess)
        he = launch_remap(d_t, int(t.size()), desc_, mp_, U_[0], halo_, nvar_, cfg_.physics == AGILE_SRHD, out_dev, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (!d_tasks) (void)hipFree(d_t);
    if (he != hipSuccess) {
        err = std::string("remap: ") + hipGetErrorString(he);
        return AGILE_EDEVICE;
    }
    return AGILE_OK;
}

int Engine::read_ghosts(int s, double *out, int out_on_device, std::string &err) {
    const MeshSlot &S = slots_[s];
    const int n = int(S.plan.n);
    const size_t per = size_t(nvar_) * CELLS, pg = size_t(6) * nvar_ * SLAB;
    const hipStream_t st = cfg_.stream;
    int e = fill_ghosts(err);
    if (e) return e;
    // U[1] is free between steps; the mesh's range there holds n * per >= n * pg doubles
    double *scratch = U_[1] + size_t(S.first) * per;
    CHK(launch_read_ghosts(desc_, U_[0], halo_, scratch, S.first, n, nvar_, st));
    if (out_on_device) {
        CHK(launch_permute(scratch, out, S.d_perm, 0, n, int(pg), 1, st));
        return AGILE_OK;
    }
    std::vector<double> tmp(size_t(n) * pg);
    CHK(hipMemcpyAsync(tmp.data(), scratch, tmp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    CHK(hipStreamSynchronize(st));
    for (int q = 0; q < n; ++q)
        std::memcpy(out + size_t(q) * pg, &tmp[size_t(S.plan.perm[q]) * pg], pg * sizeof(double));
    return AGILE_OK;
}

// Autotuner: the stage kernel's shape (planes per workgroup, XCD-aware mapping)
// changes the order in which work is scheduled but not the arithmetic of any
// cell, so every candidate gives bitwise the same result.
//
// With the engine's own memory the candidates are timed in whole steps: the
// state of every active mesh (U[0], its x-boundary copy, the per-block signal
// maxima and the mesh parameters) is copied aside, each candidate runs one
// step to warm up and three timed steps, and the state is copied back after
// each.  The first-stage shape is chosen with the last stage's fixed, then
// the last stage's (the middle SSP-RK3 stage takes the first stage's shape);
// a candidate replaces the current shape only when at least 1% faster.
// Without room for the copy (a caller-owned pool, or the device refuses it)
// single launches of each stage kind are timed on the current state instead
// (they only write the stage buffer, its boundary copy, flux registers and
// the per-block maxima, which are restored or rewritten by the next step);
// that timing does not reproduce a step's cache state, so its choice can
// differ from the whole-step optimum by a few percent.
int Engine::tune(std::string &err, int max_blocks) {
    int e = rebuild(err);
    if (e) return e;
    if (nlist_ == 0 || nvar_ == 9) return AGILE_OK;   // the MHD stage has a single shape
    const hipStream_t st = cfg_.stream;
    // copy of the state of the active meshes
    const size_t pu = size_t(nvar_) * CELLS, px = size_t(nvar_) * XE_CELLS;
    size_t nact = 0;
    for (const MeshSlot &S : slots_)
        if (S.used && S.active) nact += size_t(S.plan.n);
    const size_t nsm = size_t(cfg_.cap_blocks) * (cmax_ ? 2 : 1);
    const size_t bytes = nact * (pu + px) * sizeof(double) + nsm * sizeof(unsigned long long) +
                         size_t(cfg_.cap_meshes) * sizeof(MeshParams);
    char *save = nullptr;
    if (!owns_ || hipMalloc(&save, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return tune_launches(err, max_blocks);
    }
    auto copy_state = [&](bool back) -> hipError_t {
        char *q = save;
        hipError_t r = hipSuccess;
        auto cp = [&](void *dev, size_t nb) {
            if (r == hipSuccess)
                r = back ? hipMemcpyAsync(dev, q, nb, hipMemcpyDeviceToDevice, st)
                         : hipMemcpyAsync(q, dev, nb, hipMemcpyDeviceToDevice, st);
            q += nb;
        };
        for (const MeshSlot &S : slots_) {
            if (!(S.used && S.active)) continue;
            cp(U_[0] + size_t(S.first) * pu, size_t(S.plan.n) * pu * sizeof(double));
            cp(XE_[0] + size_t(S.first) * px, size_t(S.plan.n) * px * sizeof(double));
        }
        cp(smax_, nsm * sizeof(unsigned long long));
        cp(mp_, size_t(cfg_.cap_meshes) * sizeof(MeshParams));
        return r;
    };
    hipEvent_t t0 = nullptr, t1 = nullptr;
    const int keep_timing = timing_;
    timing_ = 0;
    auto finish = [&](int rc) {
        timing_ = keep_timing;
        if (t0) (void)hipEventDestroy(t0);
        if (t1) (void)hipEventDestroy(t1);
        (void)hipStreamSynchronize(st);
        (void)hipFree(save);
        ghosts_valid_ = false;   // the halo slabs hold the ghosts of a trial step
        dirty_ = true;           // re-capture the step graph
        return rc;
    };
    std::string e2;
    if (copy_state(false) != hipSuccess || hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess)
        return finish((err = "tuner: state copy or events failed", AGILE_EDEVICE));
    // time of 3 steps with the current shapes (after one warm-up step), the
    // state restored afterwards
    auto trial = [&](float &ms) -> int {
        ghosts_valid_ = false;
        int rc = enqueue_step(true, e2);
        if (!rc && hipEventRecord(t0, st) != hipSuccess) rc = AGILE_EDEVICE;
        for (int r = 0; r < 3 && !rc; ++r) rc = enqueue_step(true, e2);
        if (!rc && hipEventRecord(t1, st) != hipSuccess) rc = AGILE_EDEVICE;
        if (!rc && hipEventSynchronize(t1) != hipSuccess) rc = AGILE_EDEVICE;
        if (!rc && hipEventElapsedTime(&ms, t0, t1) != hipSuccess) rc = AGILE_EDEVICE;
        if (!rc && copy_state(true) != hipSuccess) rc = AGILE_EDEVICE;
        if (rc && e2.empty()) e2 = "tuner: trial step failed";
        return rc;
    };
    const int ks_c[3] = {16, 8, 4};
    for (int t = 0; t < 2; ++t) {
        int &ks_ref = t == 0 ? kslab : kslab_last, &x_ref = t == 0 ? xcd : xcd_last;
        const int ks0 = ks_ref, x0 = x_ref;   // ks0 = 0: the automatic depth
        float base = 0.f;
        int rc = trial(base);
        if (rc) {
            err = e2;
            return finish(rc);
        }
        float best = base;
        int bk = ks0, bx = x0;
        for (int ks : ks_c)
            for (int x : {0, 1}) {
                if (ks == ks0 && x == x0) continue;
                ks_ref = ks;
                x_ref = x;
                float ms = 0.f;
                if ((rc = trial(ms))) {
                    ks_ref = ks0;
                    x_ref = x0;
                    err = e2;
                    return finish(rc);
                }
                if (ms < best) {
                    best = ms;
                    bk = ks;
                    bx = x;
                }
            }
        if (best < 0.99f * base) {
            ks_ref = bk;
            x_ref = bx;
        } else {
            ks_ref = ks0;
            x_ref = x0;
        }
    }
    return finish(AGILE_OK);
}

// The single-launch form of the tuner (see above).
int Engine::tune_launches(std::string &err, int max_blocks) {
    const hipStream_t st = cfg_.stream;
    int e;
    if ((e = enqueue_fill(0, err))) return e;
    hipEvent_t t0, t1;
    CHK(hipEventCreate(&t0));
    CHK(hipEventCreate(&t1));
    // candidates in order, the current shape first: another replaces it only
    // when at least 2% faster
    const int ks_c[3] = {16, 8, 4};
    // the first stage, and the last stage of a step (SSP-RK2: kind 2,
    // SSP-RK3: kind 4; the middle stage takes the first stage's shape).
    // Every timed launch reads U[0] (as input and as U^n) and writes U[1],
    // which is free between steps: the same work as in a step, on a valid
    // state, with the mesh's state untouched.
    const int kinds[2] = {1, cfg_.rk == 3 ? 4 : 2};
    int bk[2] = {stage_kslab(false), stage_kslab(true)}, bx[2] = {xcd, xcd_last};
    for (int t = 0; t < 2; ++t) {
        float best = 1e30f;
        std::vector<std::pair<int, int>> cand{{bk[t], bx[t]}};
        for (int ks : ks_c)
            for (int x : {0, 1})
                if (ks != bk[t] || x != bx[t]) cand.push_back({ks, x});
        for (const auto &c : cand) {
            const int ks = c.first, x = c.second;
            StageArgs a{};
            a.desc = desc_;
            a.mp = mp_;
            a.halo = halo_;
            a.freg = freg_;
            a.smax = smax_;
            a.list = d_list_;
            a.nblocks = std::min(nlist_, std::max(max_blocks, 1));   // beyond a few thousand blocks the
            a.kslab = ks;                                              // per-block cost no longer changes
            a.xcd = x;
            a.stage = kinds[t];
            a.limiter = cfg_.limiter;
            a.Uin = U_[0];
            a.Uout = U_[1];
            a.Un = kinds[t] == 1 ? nullptr : U_[0];
            a.XEin = XE_[0];
            a.XEout = XE_[1];
            CHK(launch_stage(a, stage_solver(), cfg_.precision, st));
            CHK(hipEventRecord(t0, st));
            for (int r = 0; r < 3; ++r) CHK(launch_stage(a, stage_solver(), cfg_.precision, st));
            CHK(hipEventRecord(t1, st));
            CHK(hipEventSynchronize(t1));
            float ms = 0.f;
            CHK(hipEventElapsedTime(&ms, t0, t1));
            if (ms < best * 0.98f) {
                best = ms;
                bk[t] = ks;
                bx[t] = x;
            }
        }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    // restore the per-block signal maxima of the current state
    for (const MeshSlot &S : slots_)
        if (S.used && S.active) CHK(launch_smax(desc_, mp_, U_[0], smax_, cmax_, S.first, int(S.plan.n), nvar_, st));
    CHK(hipStreamSynchronize(st));
    if (bk[0] != kslab || bx[0] != xcd || bk[1] != kslab_last || bx[1] != xcd_last) {
        kslab = bk[0];
        xcd = bx[0];
        kslab_last = bk[1];
        xcd_last = bx[1];
        dirty_ = true;   // re-capture the step graph
    }
    return AGILE_OK;
}

} // namespace agile
