// agile_abi.cpp -- C-ABI entry points (include/agile.h) of the MI355X
// block-AMR library: mesh lifetime, device memory, and the order in which the
// kernels of one SSP-RK2 step are enqueued on the mesh's stream.
//
// One step (stages s = 1, 2), buffers A = U^n / U^{n+1}, B = U^(1):
//   ghost fill of A (restriction, then prolongation level by level)
//   stage 1: A -> B          flux correction of B
//   ghost fill of B
//   stage 2: (B, A) -> A     flux correction of A (+ signal rate of corrected cells)
//   dt reduction over the per-block signal maxima of A
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/agile.h"
#include "agile_internal.hpp"
#include "mesh.hpp"

namespace agile {
hipError_t launch_stage(const StageArgs &a, int riemann, int precision, hipStream_t s);
hipError_t launch_restrict(const RestrictTask *t, int n, const double *U, double *halo, int NV, hipStream_t s);
hipError_t launch_prolong(const ProlongTask *t, int n, const BlockDesc *desc, const double *U, double *halo, int NV,
                          hipStream_t s);
hipError_t launch_reflux(const RefluxTask *t, int n, const BlockDesc *desc, MeshParams *mp, double *U, double *XE,
                         const double *freg, unsigned long long *smax, int NV, int stage, hipStream_t s);
hipError_t launch_xexport(const double *U, double *XE, int nblocks, int NV, hipStream_t s);
hipError_t launch_smax(const BlockDesc *desc, MeshParams *mp, const double *U, unsigned long long *smax, int nblocks,
                       int NV, hipStream_t s);
hipError_t launch_dt_finalize(MeshParams *mp, int mesh, const unsigned long long *smax, int first, int n, int set_dt,
                              hipStream_t s);
hipError_t launch_set_dt(MeshParams *mp, int mesh, double dt, hipStream_t s);
hipError_t launch_permute(const double *src, double *dst, const int *map, int nblocks, int per_block, int gather,
                          hipStream_t s);
hipError_t launch_read_ghosts(const BlockDesc *desc, const double *U, const double *halo, double *out, int nblocks,
                              int NV, hipStream_t s);
} // namespace agile

using namespace agile;

struct agile_mesh {
    agile_config cfg{};
    int nvar = 5;
    hipStream_t stream = nullptr;
    Plan plan;
    bool ready = false;
    double *U[2] = {nullptr, nullptr};
    double *XE[2] = {nullptr, nullptr};
    double *halo = nullptr;
    double *freg = nullptr;
    BlockDesc *d_desc = nullptr;
    MeshParams *d_mp = nullptr;
    RestrictTask *d_restrict = nullptr;
    ProlongTask *d_prolong = nullptr;
    RefluxTask *d_reflux = nullptr;
    unsigned long long *d_smax = nullptr;
    int *d_perm = nullptr;   // caller index -> device index
    std::vector<int> prolong_off, prolong_cnt;
    int err = AGILE_OK;
    std::string msg;
    // kernel timing (agile_profile)
    bool timing = false;
    std::vector<hipEvent_t> events;   // pairs (start, stop)
    std::vector<int> event_kind;      // kind of each pair
    size_t pairs_used = 0;
    double ms[4] = {0, 0, 0, 0};
    int64_t launches[4] = {0, 0, 0, 0};
};

namespace {

int set_error(agile_mesh *m, int code, const std::string &msg) {
    if (m && m->err == AGILE_OK) {
        m->err = code;
        m->msg = msg;
    }
    return code;
}

#define HIPCHK(m, call)                                                                              \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess)                                                                        \
            return set_error(m, AGILE_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));   \
    } while (0)

void free_device(agile_mesh *m) {
    void *ptrs[] = {m->U[0], m->U[1], m->XE[0], m->XE[1], m->halo, m->freg, m->d_desc, m->d_mp,
                    m->d_restrict, m->d_prolong, m->d_reflux, m->d_smax, m->d_perm};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    m->U[0] = m->U[1] = m->XE[0] = m->XE[1] = m->halo = m->freg = nullptr;
    m->d_desc = nullptr;
    m->d_mp = nullptr;
    m->d_restrict = nullptr;
    m->d_prolong = nullptr;
    m->d_reflux = nullptr;
    m->d_smax = nullptr;
    m->d_perm = nullptr;
    m->ready = false;
}

int dalloc(agile_mesh *m, void **p, size_t bytes) {
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return set_error(m, AGILE_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    return AGILE_OK;
}

int check_usable(agile_mesh *m) {
    if (!m) return AGILE_EINVAL;
    if (m->err != AGILE_OK) return AGILE_ESTATE;
    if (!m->ready) return set_error(m, AGILE_ESTATE, "no blocks set");
    return AGILE_OK;
}

// event pair around a launch when timing is on
int tbegin(agile_mesh *m, int kind) {
    if (!m->timing) return AGILE_OK;
    if (m->pairs_used == m->event_kind.size()) {
        hipEvent_t a, b;
        HIPCHK(m, hipEventCreate(&a));
        HIPCHK(m, hipEventCreate(&b));
        m->events.push_back(a);
        m->events.push_back(b);
        m->event_kind.push_back(kind);
    }
    m->event_kind[m->pairs_used] = kind;
    HIPCHK(m, hipEventRecord(m->events[2 * m->pairs_used], m->stream));
    return AGILE_OK;
}
int tend(agile_mesh *m) {
    if (!m->timing) return AGILE_OK;
    HIPCHK(m, hipEventRecord(m->events[2 * m->pairs_used + 1], m->stream));
    m->pairs_used++;
    return AGILE_OK;
}
// fold recorded pairs into the totals (synchronises the stream)
int tcollect(agile_mesh *m) {
    if (m->pairs_used == 0) return AGILE_OK;
    HIPCHK(m, hipStreamSynchronize(m->stream));
    for (size_t q = 0; q < m->pairs_used; ++q) {
        float t = 0.f;
        HIPCHK(m, hipEventElapsedTime(&t, m->events[2 * q], m->events[2 * q + 1]));
        m->ms[m->event_kind[q]] += t;
        m->launches[m->event_kind[q]] += 1;
    }
    m->pairs_used = 0;
    return AGILE_OK;
}
#define TIMED(m, kind, call)                 \
    do {                                     \
        int te_ = tbegin(m, kind);           \
        if (te_) return te_;                 \
        HIPCHK(m, call);                     \
        if ((te_ = tend(m))) return te_;     \
    } while (0)

// ghost fill of state buffer `buf`: restriction, then prolongation level by level
int fill(agile_mesh *m, int buf) {
    const int NV = m->nvar;
    if (!m->plan.restrict_tasks.empty())
        TIMED(m, AGILE_K_FILL, launch_restrict(m->d_restrict, int(m->plan.restrict_tasks.size()), m->U[buf], m->halo,
                                               NV, m->stream));
    for (size_t l = 0; l < m->prolong_cnt.size(); ++l)
        if (m->prolong_cnt[l] > 0)
            TIMED(m, AGILE_K_FILL, launch_prolong(m->d_prolong + m->prolong_off[l], m->prolong_cnt[l], m->d_desc,
                                                  m->U[buf], m->halo, NV, m->stream));
    return AGILE_OK;
}

int stage(agile_mesh *m, int s) {
    StageArgs a{};
    a.desc = m->d_desc;
    a.mp = m->d_mp;
    a.nblocks = int(m->plan.n);
    a.stage = s;
    a.halo = m->halo;
    a.freg = m->freg;
    a.smax = m->d_smax;
    if (s == 1) {
        a.Uin = m->U[0];
        a.Uout = m->U[1];
        a.Un = nullptr;
        a.XEin = m->XE[0];
        a.XEout = m->XE[1];
    } else {
        a.Uin = m->U[1];
        a.Un = m->U[0];
        a.Uout = m->U[0];
        a.XEin = m->XE[1];
        a.XEout = m->XE[0];
    }
    TIMED(m, AGILE_K_STAGE, launch_stage(a, m->cfg.riemann, m->cfg.precision, m->stream));
    const int nt = int(m->plan.reflux.size());
    if (nt > 0)
        TIMED(m, AGILE_K_REFLUX, launch_reflux(m->d_reflux, nt, m->d_desc, m->d_mp, s == 1 ? m->U[1] : m->U[0],
                                               s == 1 ? m->XE[1] : m->XE[0], m->freg, m->d_smax, m->nvar, s,
                                               m->stream));
    return AGILE_OK;
}

int one_step(agile_mesh *m) {
    int e;
    if ((e = fill(m, 0))) return e;
    if ((e = stage(m, 1))) return e;
    if ((e = fill(m, 1))) return e;
    if ((e = stage(m, 2))) return e;
    TIMED(m, AGILE_K_DT, launch_dt_finalize(m->d_mp, 0, m->d_smax, 0, int(m->plan.n), 0, m->stream));
    return AGILE_OK;
}

int read_params(agile_mesh *m, MeshParams &hp) {
    HIPCHK(m, hipMemcpyAsync(&hp, m->d_mp, sizeof(MeshParams), hipMemcpyDeviceToHost, m->stream));
    HIPCHK(m, hipStreamSynchronize(m->stream));
    return AGILE_OK;
}

int check_flags(agile_mesh *m, MeshParams &hp) {
    int e = read_params(m, hp);
    if (e) return e;
    if (hp.flags & 1) return set_error(m, AGILE_ENONPHYSICAL, "non-physical state (rho <= 0, p <= 0 or NaN)");
    return AGILE_OK;
}

} // namespace

extern "C" {

const char *agile_strerror(int code) {
    switch (code) {
    case AGILE_OK: return "ok";
    case AGILE_EINVAL: return "invalid argument";
    case AGILE_ENOMEM: return "out of memory";
    case AGILE_EDEVICE: return "device error";
    case AGILE_ESTATE: return "invalid state";
    case AGILE_ENONPHYSICAL: return "non-physical state";
    default: return "unknown error";
    }
}

const char *agile_last_error(const agile_mesh *m) { return m ? m->msg.c_str() : ""; }

static int check_config(const agile_config *cfg) {
    if (cfg->block_n != BN || cfg->nghost != NG) return AGILE_EINVAL;
    if (cfg->physics != AGILE_EULER) return AGILE_EINVAL;
    if (cfg->riemann != AGILE_HLL && cfg->riemann != AGILE_HLLC) return AGILE_EINVAL;
    if (cfg->precision != AGILE_FP64 && cfg->precision != AGILE_FP32_FLUX) return AGILE_EINVAL;
    if (!(cfg->gamma > 1.0) || !(cfg->cfl > 0.0)) return AGILE_EINVAL;
    if (cfg->max_level < 1 || cfg->max_level > MAXLEV) return AGILE_EINVAL;
    double dx[3];
    for (int d = 0; d < 3; ++d) {
        if (cfg->base_blocks[d] < 1 || !(cfg->hi[d] > cfg->lo[d])) return AGILE_EINVAL;
        dx[d] = (cfg->hi[d] - cfg->lo[d]) / (double(cfg->base_blocks[d]) * BN);
    }
    for (int d = 1; d < 3; ++d)
        if (std::fabs(dx[d] - dx[0]) > 1e-14 * dx[0]) return AGILE_EINVAL;
    return AGILE_OK;
}

int agile_plan(const agile_config *cfg, int64_t nblocks, const agile_block_desc *blocks, agile_plan_stats *out,
               char *msg, int msg_len) {
    auto put = [&](const std::string &s) {
        if (msg && msg_len > 0) {
            std::strncpy(msg, s.c_str(), size_t(msg_len) - 1);
            msg[msg_len - 1] = 0;
        }
    };
    if (!cfg || check_config(cfg) != AGILE_OK) {
        put("invalid config");
        return AGILE_EINVAL;
    }
    Plan P;
    PlanInput in{{cfg->base_blocks[0], cfg->base_blocks[1], cfg->base_blocks[2]}, cfg->max_level};
    if (build_plan(in, nblocks, blocks, P) != AGILE_OK) {
        put(P.error);
        return AGILE_EINVAL;
    }
    put("");
    if (out) {
        const int nvar = cfg->physics == AGILE_EULER ? 5 : 9;
        agile_plan_stats st{};
        st.nblocks = P.n;
        for (const BlockDesc &D : P.desc)
            for (int f = 0; f < 6; ++f) st.same_level_faces += D.nb[f] >= 0;
        st.restrict_tasks = int64_t(P.restrict_tasks.size());
        for (const auto &v : P.prolong) st.prolong_tasks += int64_t(v.size());
        st.reflux_blocks = int64_t(P.reflux.size());
        st.flux_registers = P.nfreg;
        st.levels = P.levels;
        st.nvar = nvar;
        st.device_bytes = int64_t(plan_device_bytes(P, nvar));
        *out = st;
    }
    return AGILE_OK;
}

int agile_mesh_create(const agile_config *cfg, agile_mesh **out) {
    if (!cfg || !out) return AGILE_EINVAL;
    if (check_config(cfg) != AGILE_OK) return AGILE_EINVAL;
    agile_mesh *m = new (std::nothrow) agile_mesh();
    if (!m) return AGILE_ENOMEM;
    m->cfg = *cfg;
    m->nvar = 5;
    m->stream = reinterpret_cast<hipStream_t>(cfg->stream);
    *out = m;
    return AGILE_OK;
}

int agile_set_blocks(agile_mesh *m, int64_t nblocks, const agile_block_desc *blocks, const double *u,
                     int u_on_device) {
    if (!m) return AGILE_EINVAL;
    if (m->err != AGILE_OK) return AGILE_ESTATE;
    if (!u) return set_error(m, AGILE_EINVAL, "null state");
    Plan P;
    PlanInput in{{m->cfg.base_blocks[0], m->cfg.base_blocks[1], m->cfg.base_blocks[2]}, m->cfg.max_level};
    if (build_plan(in, nblocks, blocks, P) != AGILE_OK) return set_error(m, AGILE_EINVAL, P.error);
    if (m->ready) HIPCHK(m, hipStreamSynchronize(m->stream));
    free_device(m);
    m->plan = std::move(P);
    const Plan &p = m->plan;
    const int NV = m->nvar;
    const size_t n = size_t(p.n);
    int e;
    for (int s = 0; s < 2; ++s) {
        if ((e = dalloc(m, (void **)&m->U[s], n * NV * CELLS * sizeof(double)))) return e;
        if ((e = dalloc(m, (void **)&m->XE[s], n * NV * XE_CELLS * sizeof(double)))) return e;
    }
    if ((e = dalloc(m, (void **)&m->halo, size_t(p.nhalo) * NV * SLAB * sizeof(double)))) return e;
    if ((e = dalloc(m, (void **)&m->freg, size_t(p.nfreg) * NV * REG * sizeof(double)))) return e;
    if ((e = dalloc(m, (void **)&m->d_desc, n * sizeof(BlockDesc)))) return e;
    if ((e = dalloc(m, (void **)&m->d_mp, sizeof(MeshParams)))) return e;
    if ((e = dalloc(m, (void **)&m->d_smax, n * sizeof(unsigned long long)))) return e;
    if ((e = dalloc(m, (void **)&m->d_perm, n * sizeof(int)))) return e;
    std::vector<ProlongTask> pro;
    m->prolong_off.assign(p.prolong.size(), 0);
    m->prolong_cnt.assign(p.prolong.size(), 0);
    for (size_t l = 0; l < p.prolong.size(); ++l) {
        m->prolong_off[l] = int(pro.size());
        m->prolong_cnt[l] = int(p.prolong[l].size());
        pro.insert(pro.end(), p.prolong[l].begin(), p.prolong[l].end());
    }
    if ((e = dalloc(m, (void **)&m->d_restrict, p.restrict_tasks.size() * sizeof(RestrictTask)))) return e;
    if ((e = dalloc(m, (void **)&m->d_prolong, pro.size() * sizeof(ProlongTask)))) return e;
    if ((e = dalloc(m, (void **)&m->d_reflux, p.reflux.size() * sizeof(RefluxTask)))) return e;

    MeshParams hp{};
    hp.gamma = m->cfg.gamma;
    hp.cfl = m->cfg.cfl;
    hp.inv_dx1 = (double(m->cfg.base_blocks[0]) * BN) / (m->cfg.hi[0] - m->cfg.lo[0]);
    hp.glm_alpha = m->cfg.glm_alpha;
    hp.dt = 0.0;
    hp.first_block = 0;
    hp.flags = 0;
    hipStream_t st = m->stream;
    HIPCHK(m, hipMemcpyAsync(m->d_desc, p.desc.data(), n * sizeof(BlockDesc), hipMemcpyHostToDevice, st));
    HIPCHK(m, hipMemcpyAsync(m->d_mp, &hp, sizeof(MeshParams), hipMemcpyHostToDevice, st));
    HIPCHK(m, hipMemcpyAsync(m->d_perm, p.perm.data(), n * sizeof(int), hipMemcpyHostToDevice, st));
    if (!p.restrict_tasks.empty())
        HIPCHK(m, hipMemcpyAsync(m->d_restrict, p.restrict_tasks.data(), p.restrict_tasks.size() * sizeof(RestrictTask),
                                 hipMemcpyHostToDevice, st));
    if (!pro.empty())
        HIPCHK(m, hipMemcpyAsync(m->d_prolong, pro.data(), pro.size() * sizeof(ProlongTask), hipMemcpyHostToDevice, st));
    if (!p.reflux.empty())
        HIPCHK(m, hipMemcpyAsync(m->d_reflux, p.reflux.data(), p.reflux.size() * sizeof(RefluxTask),
                                 hipMemcpyHostToDevice, st));
    const size_t per = size_t(NV) * CELLS;
    if (u_on_device) {
        HIPCHK(m, launch_permute(u, m->U[0], m->d_perm, int(n), int(per), 0, st));
    } else {
        std::vector<double> tmp(n * per);
        for (size_t q = 0; q < n; ++q) std::memcpy(&tmp[size_t(p.perm[q]) * per], u + q * per, per * sizeof(double));
        HIPCHK(m, hipMemcpyAsync(m->U[0], tmp.data(), tmp.size() * sizeof(double), hipMemcpyHostToDevice, st));
        HIPCHK(m, hipStreamSynchronize(st));
    }
    // tables must be on the device before the host vectors go out of scope
    HIPCHK(m, hipStreamSynchronize(st));
    HIPCHK(m, launch_xexport(m->U[0], m->XE[0], int(n), NV, st));
    HIPCHK(m, launch_smax(m->d_desc, m->d_mp, m->U[0], m->d_smax, int(n), NV, st));
    HIPCHK(m, launch_dt_finalize(m->d_mp, 0, m->d_smax, 0, int(n), 0, st));
    m->ready = true;
    return AGILE_OK;
}

int agile_fill_ghosts(agile_mesh *m) {
    int e = check_usable(m);
    if (e) return e;
    return fill(m, 0);
}

int agile_dt(agile_mesh *m, double *dt_out) {
    int e = check_usable(m);
    if (e) return e;
    if (!dt_out) return set_error(m, AGILE_EINVAL, "null dt_out");
    MeshParams hp;
    if ((e = check_flags(m, hp))) return e;
    double s;
    std::memcpy(&s, &hp.smax, sizeof(double));
    *dt_out = m->cfg.cfl / s;
    return AGILE_OK;
}

int agile_step(agile_mesh *m, double dt) {
    int e = check_usable(m);
    if (e) return e;
    if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(m, AGILE_EINVAL, "dt must be positive and finite");
    HIPCHK(m, launch_set_dt(m->d_mp, 0, dt, m->stream));
    if ((e = one_step(m))) return e;
    if (m->pairs_used > 4096) return tcollect(m);
    return AGILE_OK;
}

int agile_step_cfl(agile_mesh *m, int nsteps) {
    int e = check_usable(m);
    if (e) return e;
    if (nsteps < 0) return set_error(m, AGILE_EINVAL, "nsteps must be >= 0");
    for (int q = 0; q < nsteps; ++q) {
        // dt of this step from the signal maximum of its start state
        TIMED(m, AGILE_K_DT, launch_dt_finalize(m->d_mp, 0, m->d_smax, 0, int(m->plan.n), 1, m->stream));
        if ((e = one_step(m))) return e;
        if (m->pairs_used > 4096 && (e = tcollect(m))) return e;
    }
    return AGILE_OK;
}

int agile_last_dt(agile_mesh *m, double *dt_out) {
    int e = check_usable(m);
    if (e) return e;
    if (!dt_out) return set_error(m, AGILE_EINVAL, "null dt_out");
    MeshParams hp;
    if ((e = read_params(m, hp))) return e;
    *dt_out = hp.dt;
    return AGILE_OK;
}

int agile_readback(agile_mesh *m, double *u_out, int64_t capacity_doubles, int out_on_device) {
    int e = check_usable(m);
    if (e) return e;
    const size_t n = size_t(m->plan.n), per = size_t(m->nvar) * CELLS;
    if (!u_out || capacity_doubles < int64_t(n * per)) return set_error(m, AGILE_EINVAL, "output too small");
    MeshParams hp;
    if ((e = check_flags(m, hp))) return e;
    if (out_on_device) {
        HIPCHK(m, launch_permute(m->U[0], u_out, m->d_perm, int(n), int(per), 1, m->stream));
        return AGILE_OK;
    }
    std::vector<double> tmp(n * per);
    HIPCHK(m, hipMemcpyAsync(tmp.data(), m->U[0], tmp.size() * sizeof(double), hipMemcpyDeviceToHost, m->stream));
    HIPCHK(m, hipStreamSynchronize(m->stream));
    for (size_t q = 0; q < n; ++q) std::memcpy(u_out + q * per, &tmp[size_t(m->plan.perm[q]) * per], per * sizeof(double));
    return AGILE_OK;
}

int agile_read_ghosts(agile_mesh *m, double *g_out, int64_t capacity_doubles, int out_on_device) {
    int e = check_usable(m);
    if (e) return e;
    const size_t n = size_t(m->plan.n), per = size_t(6) * m->nvar * SLAB;
    if (!g_out || capacity_doubles < int64_t(n * per)) return set_error(m, AGILE_EINVAL, "output too small");
    if ((e = fill(m, 0))) return e;
    // U[1] is free between steps and holds n * nvar * 4096 >= n * 6 * nvar * 512 doubles
    HIPCHK(m, launch_read_ghosts(m->d_desc, m->U[0], m->halo, m->U[1], int(n), m->nvar, m->stream));
    if (out_on_device) {
        HIPCHK(m, launch_permute(m->U[1], g_out, m->d_perm, int(n), int(per), 1, m->stream));
        return AGILE_OK;
    }
    std::vector<double> tmp(n * per);
    HIPCHK(m, hipMemcpyAsync(tmp.data(), m->U[1], tmp.size() * sizeof(double), hipMemcpyDeviceToHost, m->stream));
    HIPCHK(m, hipStreamSynchronize(m->stream));
    for (size_t q = 0; q < n; ++q) std::memcpy(g_out + q * per, &tmp[size_t(m->plan.perm[q]) * per], per * sizeof(double));
    return AGILE_OK;
}

int agile_profile(agile_mesh *m, int enable) {
    if (!m) return AGILE_EINVAL;
    if (m->err != AGILE_OK) return AGILE_ESTATE;
    int e = tcollect(m);
    if (e) return e;
    m->timing = enable != 0;
    for (int k = 0; k < 4; ++k) {
        m->ms[k] = 0.0;
        m->launches[k] = 0;
    }
    return AGILE_OK;
}

int agile_profile_read(agile_mesh *m, int kind, double *ms_total, int64_t *launches) {
    if (!m || kind < 0 || kind > 3) return AGILE_EINVAL;
    if (m->err != AGILE_OK) return AGILE_ESTATE;
    int e = tcollect(m);
    if (e) return e;
    if (ms_total) *ms_total = m->ms[kind];
    if (launches) *launches = m->launches[kind];
    return AGILE_OK;
}

int agile_mesh_info(const agile_mesh *m, int64_t *nblocks, int *nvar) {
    if (!m) return AGILE_EINVAL;
    if (nblocks) *nblocks = m->ready ? m->plan.n : 0;
    if (nvar) *nvar = m->nvar;
    return AGILE_OK;
}

void agile_mesh_destroy(agile_mesh *m) {
    if (!m) return;
    if (m->ready) (void)hipStreamSynchronize(m->stream);
    for (hipEvent_t ev : m->events) (void)hipEventDestroy(ev);
    free_device(m);
    delete m;
}

} // extern "C"
