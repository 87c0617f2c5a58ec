// agile_abi.cpp -- C-ABI entry points (include/agile.h).
//
// agile_mesh: one mesh in an engine sized exactly for it.
// agile_batch: a serving front end over one engine whose pool is sized from an
// HBM budget: requests queue in arrival order, are admitted first-come
// first-served whenever their footprint fits (continuous batching: a request
// that arrives while others run joins at the next tick), every resident mesh
// advances one CFL step per tick in one batched launch sequence, finished
// meshes keep their state until collected.
//
// One step (stages s = 1, 2), buffers A = U^n / U^{n+1}, B = U^(1):
//   dt from the signal maximum (CFL steps), ghost fill of A, stage 1 A -> B,
//   flux correction of B, ghost fill of B, stage 2 (B, A) -> A, flux
//   correction of A, per-mesh signal maximum and time.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/agile.h"
#include "agile_internal.hpp"
#include "engine.hpp"
#include "mesh.hpp"

using namespace agile;

namespace agile {
RemapTask *noalloc_scratch(int device, std::string &err);   // noalloc.hip
}

namespace {

int check_config(const agile_config *cfg) {
    if (!cfg) return AGILE_EINVAL;
    if ((cfg->block_n != BN && cfg->block_n != 2 * BN && cfg->block_n != 4 * BN) || cfg->nghost != NG)
        return AGILE_EINVAL;
    if (cfg->physics != AGILE_EULER && cfg->physics != AGILE_MHD_GLM && cfg->physics != AGILE_SRHD) return AGILE_EINVAL;
    if (cfg->physics == AGILE_SRHD && cfg->riemann != AGILE_LF) return AGILE_EINVAL;   // SRHD: LF (Table 1)
    if (cfg->riemann != AGILE_HLL && cfg->riemann != AGILE_HLLC && cfg->riemann != AGILE_LF) return AGILE_EINVAL;
    if (cfg->limiter != AGILE_MINMOD && cfg->limiter != AGILE_VANLEER) return AGILE_EINVAL;
    if (cfg->rk_stages != 0 && cfg->rk_stages != 2 && cfg->rk_stages != 3) return AGILE_EINVAL;
    if (cfg->physics == AGILE_MHD_GLM && (cfg->riemann != AGILE_HLL || !(cfg->glm_alpha >= 0.0) ||
                                          cfg->limiter != AGILE_MINMOD || cfg->rk_stages == 3))
        return AGILE_EINVAL;   // MHD: HLL (Table 1), minmod, SSP-RK2
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
    if (cfg->dev_pool && cfg->dev_pool_bytes == 0) return AGILE_EINVAL;
    return AGILE_OK;
}

// Engine config of a single mesh whose plan is P: the scheme of cfg, room for
// `headroom` times the plan's blocks, ghost slabs and flux registers.  With a
// caller pool, as much room as the pool holds (each block beyond the plan's
// with 1.5 ghost slabs and flux registers), AGILE_ENOMEM when not even the
// plan fits.
int mesh_engine_config(const agile_config &cfg, const Plan &P, double headroom, EngineConfig &ec, std::string &err) {
    ec = EngineConfig{};
    ec.physics = cfg.physics;
    ec.riemann = cfg.riemann;
    ec.precision = cfg.precision;
    ec.limiter = cfg.limiter;
    ec.rk = cfg.rk_stages == 3 ? 3 : 2;
    ec.stream = reinterpret_cast<hipStream_t>(cfg.stream);
    ec.cap_meshes = 1;
    auto caps = [&](double h) {
        const double extra = double(P.n) * (h - 1.0);
        ec.cap_blocks = int(std::max<int64_t>(1, int64_t(std::ceil(double(P.n) * h))));
        ec.cap_halo = int(P.nhalo + int64_t(1.5 * extra));
        ec.cap_freg = int(P.nfreg + int64_t(1.5 * extra));
    };
    if (!cfg.dev_pool) {
        ec.cap_blocks = int(std::max<int64_t>(1, int64_t(double(P.n) * headroom)));
        ec.cap_halo = int(double(P.nhalo) * headroom);
        ec.cap_freg = int(double(P.nfreg) * headroom);
        return AGILE_OK;
    }
    ec.pool = cfg.dev_pool;
    ec.pool_bytes = cfg.dev_pool_bytes;
    caps(1.0);
    const size_t need = engine_device_bytes(ec);
    if (need > cfg.dev_pool_bytes) {
        err = "caller device pool too small: " + std::to_string(cfg.dev_pool_bytes) + " bytes given, " +
              std::to_string(need) + " needed";
        return AGILE_ENOMEM;
    }
    double lo = 1.0, hi = 2.0;   // largest headroom that still fits (bisection)
    for (caps(hi); engine_device_bytes(ec) <= cfg.dev_pool_bytes && hi < double(1 << 20); caps(hi)) hi *= 2.0;
    for (int it = 0; it < 40; ++it) {
        const double mid = 0.5 * (lo + hi);
        caps(mid);
        (engine_device_bytes(ec) <= cfg.dev_pool_bytes ? lo : hi) = mid;
    }
    caps(lo);
    if (int64_t(ec.cap_blocks) > (int64_t(1) << 30)) ec.cap_blocks = 1 << 30;
    return AGILE_OK;
}

// A block of block_n = 16 te cells per edge is stored and updated as te^3
// tiles of 16^3 cells: the tile mesh has te times the base blocks per axis,
// the same levels, and its tiles in block order (sub-tile x fastest).
int tile_edge(const agile_config &cfg) { return cfg.block_n / BN; }

agile_config tile_config(const agile_config &cfg) {
    agile_config t = cfg;
    const int te = tile_edge(cfg);
    t.block_n = BN;
    for (int d = 0; d < 3; ++d) t.base_blocks[d] = cfg.base_blocks[d] * te;
    return t;
}

std::vector<agile_block_desc> expand_tiles(int64_t n, const agile_block_desc *blocks, int te) {
    std::vector<agile_block_desc> t;
    t.reserve(size_t(n) * te * te * te);
    for (int64_t q = 0; q < n; ++q)
        for (int z = 0; z < te; ++z)
            for (int y = 0; y < te; ++y)
                for (int x = 0; x < te; ++x)
                    t.push_back(agile_block_desc{blocks[q].level,
                                                 {blocks[q].idx[0] * te + x, blocks[q].idx[1] * te + y,
                                                  blocks[q].idx[2] * te + z}});
    return t;
}

// Validate a block list at block granularity, then plan its 16^3 tiles.
int plan_blocks(const agile_config &cfg, int64_t n, const agile_block_desc *blocks, Plan &P) {
    PlanInput in{{cfg.base_blocks[0], cfg.base_blocks[1], cfg.base_blocks[2]}, cfg.max_level};
    if (build_plan(in, n, blocks, P) != AGILE_OK) return AGILE_EINVAL;
    const int te = tile_edge(cfg);
    if (te == 1) return AGILE_OK;
    const std::vector<agile_block_desc> t = expand_tiles(n, blocks, te);
    const agile_config tc = tile_config(cfg);
    PlanInput ti{{tc.base_blocks[0], tc.base_blocks[1], tc.base_blocks[2]}, tc.max_level};
    return build_plan(ti, int64_t(t.size()), t.data(), P);
}

void put_msg(char *msg, int len, const std::string &s) {
    if (msg && len > 0) {
        std::strncpy(msg, s.c_str(), size_t(len) - 1);
        msg[len - 1] = 0;
    }
}

} // namespace

struct agile_mesh {
    agile_config cfg{};
    int nvar = 5;
    std::unique_ptr<Engine> eng;
    int slot = -1;
    int err = AGILE_OK;
    std::string msg;
    int use_graph = 0, kslab = 0, xcd = 0, kslab_last = 0, xcd_last = 0;
    int device = -1;                        // device current at agile_set_blocks
    int te = 1;                             // 16^3 tiles per block edge
    agile_config tcfg{};                    // the config of the tile mesh
    std::vector<agile_block_desc> blocks;   // current leaves, caller's order
};

struct agile_batch {
    agile_batch_config cfg{};
    std::unique_ptr<Engine> eng;
    struct Request {
        agile_config cfg;
        Plan plan;
        std::vector<agile_block_desc> blocks;   // its leaves, in the order of its state
        std::vector<double> u;        // host copy, or
        const double *dev = nullptr;  // the caller's device buffer (read at admission)
        int64_t steps;
        uint64_t tag;
        int64_t done = 0;             // steps taken before a regrid sent it back to the queue
        bool has_carry = false;       // time, dt and flags of that earlier residence
        MeshParams carry{};
    };
    std::deque<Request> queue;
    std::map<uint64_t, int> resident;          // tag -> engine slot
    std::map<uint64_t, std::vector<agile_block_desc>> res_blocks;   // tag -> leaves of a resident request
    std::map<int, std::array<int, 4>> tuned;  // active-block size class -> (kslab, xcd, kslab_last, xcd_last)
    int err = AGILE_OK;
    std::string msg;
};

namespace {

int fail(agile_mesh *m, int code, const std::string &msg) {
    if (m && m->err == AGILE_OK) {
        m->err = code;
        m->msg = msg;
    }
    return code;
}
int fail(agile_batch *b, int code, const std::string &msg) {
    if (b && b->err == AGILE_OK) {
        b->err = code;
        b->msg = msg;
    }
    return code;
}

// A refusal that leaves the mesh as it was: the code is returned and the
// reason kept for agile_last_error, but no sticky error is set.
int refuse(agile_mesh *m, int code, const std::string &msg) {
    if (m && m->err == AGILE_OK) m->msg = msg;
    return code;
}

int usable(agile_mesh *m) {
    if (!m) return AGILE_EINVAL;
    if (m->err != AGILE_OK) return AGILE_ESTATE;
    if (!m->eng) return fail(m, AGILE_ESTATE, "no blocks set");
    return AGILE_OK;
}

// No C++ exception may leave an extern "C" entry point: a failed host
// allocation becomes AGILE_ENOMEM, anything else AGILE_EDEVICE, recorded as the
// handle's sticky error when there is a handle.
template <class H, class F>
int guarded(H *h, F &&body) noexcept {
    int code = AGILE_EDEVICE;
    const char *what = "internal error";
    try {
        return body();
    } catch (const std::bad_alloc &) {
        code = AGILE_ENOMEM;
        what = "host allocation failed";
    } catch (...) {
    }
    try {
        return fail(h, code, what);
    } catch (...) {
        if (h && h->err == AGILE_OK) h->err = code;
        return code;
    }
}

int mesh_flags(agile_mesh *m, MeshParams &hp) {
    std::string e;
    int rc = m->eng->read_params(m->slot, hp, e);
    if (rc) return fail(m, rc, e);
    if (hp.flags & 1) return fail(m, AGILE_ENONPHYSICAL, "non-physical state (rho <= 0, p <= 0 or NaN)");
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

int agile_plan(const agile_config *cfg, int64_t nblocks, const agile_block_desc *blocks, agile_plan_stats *out,
               char *msg, int msg_len) {
    return guarded(static_cast<agile_mesh *>(nullptr), [&]() -> int {
        if (check_config(cfg) != AGILE_OK) {
            put_msg(msg, msg_len, "invalid config");
            return AGILE_EINVAL;
        }
        Plan P;
        if (plan_blocks(*cfg, nblocks, blocks, P) != AGILE_OK) {
            put_msg(msg, msg_len, P.error);
            return AGILE_EINVAL;
        }
        put_msg(msg, msg_len, "");
        if (out) {
            const int nvar = cfg->physics == AGILE_MHD_GLM ? 9 : 5;
            agile_plan_stats st{};
            st.nblocks = nblocks;
            for (const BlockDesc &D : P.desc)
                for (int f = 0; f < 6; ++f) st.same_level_faces += D.nb[f] >= 0;
            st.restrict_tasks = int64_t(P.restrict_tasks.size());
            for (const auto &v : P.prolong) st.prolong_tasks += int64_t(v.size());
            st.reflux_blocks = int64_t(P.reflux.size());
            st.flux_registers = P.nfreg;
            st.levels = P.levels;
            st.nvar = nvar;
            {
                agile_config c1 = *cfg;
                c1.dev_pool = nullptr;
                EngineConfig ec;
                std::string e;
                (void)mesh_engine_config(c1, P, 1.0, ec, e);
                st.device_bytes = int64_t(engine_device_bytes(ec));
            }
            int count = 0;
            for (size_t l = 0; l < P.prolong.size(); ++l) {
                if (P.prolong[l].empty()) continue;
                if (P.prolong_dep[l] && count > 0) {
                    st.prolong_launches++;
                    count = 0;
                }
                count += int(P.prolong[l].size());
            }
            if (count > 0) st.prolong_launches++;
            {
                std::vector<char> corrected(size_t(P.n), 0);
                for (const RefluxTask &r : P.reflux) corrected[r.block] = 1;
                st.fused_correction = 1;
                for (const RestrictTask &t : P.restrict_tasks)
                    for (int q = 0; q < 4; ++q)
                        if (corrected[t.fine[q]]) st.fused_correction = 0;
            }
            *out = st;
        }
        return AGILE_OK;
    });
}

// ---------------------------------------------------------------------------
// single mesh

int agile_mesh_create(const agile_config *cfg, agile_mesh **out) {
    return guarded(static_cast<agile_mesh *>(nullptr), [&]() -> int {
        if (!out || check_config(cfg) != AGILE_OK) return AGILE_EINVAL;
        agile_mesh *m = new (std::nothrow) agile_mesh();
        if (!m) return AGILE_ENOMEM;
        m->cfg = *cfg;
        m->nvar = cfg->physics == AGILE_MHD_GLM ? 9 : 5;
        m->te = tile_edge(*cfg);
        m->tcfg = tile_config(*cfg);
        *out = m;
        return AGILE_OK;
    });
}

namespace {

// New engine for the mesh with a plan; headroom > 1 sizes the pool for a
// larger mesh to come (regrids) so that it can be reused.
// P is the plan of the 16^3 tiles of `blocks`; u holds blocks (u_edge = te)
// or tiles (u_edge = 1).
int new_engine(agile_mesh *m, Plan &&P, int64_t nblocks, const agile_block_desc *blocks, const double *u,
               int u_on_device, double headroom, const MeshParams *carry = nullptr, int u_edge = -1) {
    if (u_edge < 0) u_edge = m->te;
    if (m->eng) (void)hipStreamSynchronize(m->eng->stream());
    m->eng.reset();
    m->slot = -1;
    EngineConfig ec;
    std::string e0;
    int rc0 = mesh_engine_config(m->tcfg, P, headroom, ec, e0);
    if (rc0) return fail(m, rc0, e0);
    std::unique_ptr<Engine> eng(new (std::nothrow) Engine());
    if (!eng) return fail(m, AGILE_ENOMEM, "host allocation failed");
    std::string e;
    int rc = eng->init(ec, e);
    if (rc) return fail(m, rc, e);
    if (hipGetDevice(&m->device) != hipSuccess) return fail(m, AGILE_EDEVICE, "no current device");
    eng->use_graph = m->use_graph != 0;
    eng->kslab = m->kslab;
    eng->xcd = m->xcd;
    eng->kslab_last = m->kslab_last;
    eng->xcd_last = m->xcd_last;
    int slot = -1;
    rc = eng->add(m->tcfg, std::move(P), u, u_on_device, -1, 0, &slot, e, carry, u_edge, m->te);
    if (rc) return fail(m, rc, e);
    m->eng = std::move(eng);
    m->slot = slot;
    m->blocks.assign(blocks, blocks + nblocks);
    return AGILE_OK;
}

} // namespace

int agile_set_blocks(agile_mesh *m, int64_t nblocks, const agile_block_desc *blocks, const double *u,
                     int u_on_device) {
    return guarded(m, [&]() -> int {
        if (!m) return AGILE_EINVAL;
        if (m->err != AGILE_OK) return AGILE_ESTATE;
        if (!u) return fail(m, AGILE_EINVAL, "null state");
        Plan P;
        if (plan_blocks(m->cfg, nblocks, blocks, P) != AGILE_OK) return fail(m, AGILE_EINVAL, P.error);
        return new_engine(m, std::move(P), nblocks, blocks, u, u_on_device, 1.0);
    });
}

int agile_mesh_set_option(agile_mesh *m, int option, int value) {
    return guarded(m, [&]() -> int {
        if (!m) return AGILE_EINVAL;
        if (m->err != AGILE_OK) return AGILE_ESTATE;
        switch (option) {
        case AGILE_OPT_GRAPH: m->use_graph = value != 0; break;
        case AGILE_OPT_KSLAB:
        case AGILE_OPT_KSLAB_LAST:
            if (value != 0 && value != 16 && value != 8 && value != 4) return AGILE_EINVAL;
            if (option == AGILE_OPT_KSLAB) m->kslab = value;
            m->kslab_last = value;
            break;
        case AGILE_OPT_XCD: m->xcd = m->xcd_last = value != 0; break;
        case AGILE_OPT_XCD_LAST: m->xcd_last = value != 0; break;
        default: return AGILE_EINVAL;
        }
        if (m->eng) {
            const bool shape = m->eng->kslab != m->kslab || m->eng->xcd != m->xcd ||
                               m->eng->kslab_last != m->kslab_last || m->eng->xcd_last != m->xcd_last;
            m->eng->use_graph = m->use_graph != 0;
            m->eng->kslab = m->kslab;
            m->eng->xcd = m->xcd;
            m->eng->kslab_last = m->kslab_last;
            m->eng->xcd_last = m->xcd_last;
            if (shape) {   // a captured step graph holds the old shape: rebuild it
                m->eng->set_active(m->slot, false);
                m->eng->set_active(m->slot, true);
            }
        }
        return AGILE_OK;
    });
}

int agile_mesh_get_option(const agile_mesh *m, int option, int *value) {
    return guarded(static_cast<agile_mesh *>(nullptr), [&]() -> int {
        if (!m || !value) return AGILE_EINVAL;
        switch (option) {
        case AGILE_OPT_GRAPH: *value = m->eng ? int(m->eng->use_graph) : m->use_graph; break;
        case AGILE_OPT_KSLAB: *value = m->eng ? m->eng->kslab : m->kslab; break;
        case AGILE_OPT_XCD: *value = m->eng ? m->eng->xcd : m->xcd; break;
        case AGILE_OPT_KSLAB_LAST: *value = m->eng ? m->eng->kslab_last : m->kslab_last; break;
        case AGILE_OPT_XCD_LAST: *value = m->eng ? m->eng->xcd_last : m->xcd_last; break;
        default: return AGILE_EINVAL;
        }
        return AGILE_OK;
    });
}

int agile_mesh_tune(agile_mesh *m) {
    return guarded(m, [&]() -> int {
        int e = usable(m);
        if (e) return e;
        std::string s;
        int rc = m->eng->tune(s);
        if (rc) return fail(m, rc, s);
        m->kslab = m->eng->kslab;
        m->xcd = m->eng->xcd;
        m->kslab_last = m->eng->kslab_last;
        m->xcd_last = m->eng->xcd_last;
        return AGILE_OK;
    });
}

int agile_fill_ghosts(agile_mesh *m) {
    return guarded(m, [&]() -> int {
        int e = usable(m);
        if (e) return e;
        std::string s;
        int rc = m->eng->fill_ghosts(s);
        return rc ? fail(m, rc, s) : AGILE_OK;
    });
}

int agile_dt(agile_mesh *m, double *dt_out) {
    return guarded(m, [&]() -> int {
        int e = usable(m);
        if (e) return e;
        if (!dt_out) return fail(m, AGILE_EINVAL, "null dt_out");
        MeshParams hp;
        if ((e = mesh_flags(m, hp))) return e;
        double s;
        std::memcpy(&s, &hp.smax, sizeof(double));
        *dt_out = m->cfg.cfl / s;
        return AGILE_OK;
    });
}

int agile_step(agile_mesh *m, double dt) {
    return guarded(m, [&]() -> int {
        int e = usable(m);
        if (e) return e;
        if (!(dt > 0.0) || !std::isfinite(dt)) return fail(m, AGILE_EINVAL, "dt must be positive and finite");
        std::string s;
        int rc = m->eng->step_dt(m->slot, dt, s);
        return rc ? fail(m, rc, s) : AGILE_OK;
    });
}

int agile_step_cfl(agile_mesh *m, int nsteps) {
    return guarded(m, [&]() -> int {
        int e = usable(m);
        if (e) return e;
        if (nsteps < 0) return fail(m, AGILE_EINVAL, "nsteps must be >= 0");
        std::string s;
        int rc = m->eng->step_cfl(nsteps, s);
        return rc ? fail(m, rc, s) : AGILE_OK;
    });
}

int agile_last_dt(agile_mesh *m, double *dt_out) {
    return guarded(m, [&]() -> int {
        int e = usable(m);
        if (e) return e;
        if (!dt_out) return fail(m, AGILE_EINVAL, "null dt_out");
        MeshParams hp;
        std::string s;
        int rc = m->eng->read_params(m->slot, hp, s);
        if (rc) return fail(m, rc, s);
        *dt_out = hp.dt;
        return AGILE_OK;
    });
}

int agile_mesh_time(agile_mesh *m, double *t_out) {
    return guarded(m, [&]() -> int {
        int e = usable(m);
        if (e) return e;
        if (!t_out) return fail(m, AGILE_EINVAL, "null t_out");
        MeshParams hp;
        std::string s;
        int rc = m->eng->read_params(m->slot, hp, s);
        if (rc) return fail(m, rc, s);
        *t_out = hp.t;
        return AGILE_OK;
    });
}

int agile_readback(agile_mesh *m, double *u_out, int64_t capacity_doubles, int out_on_device) {
    return guarded(m, [&]() -> int {
        int e = usable(m);
        if (e) return e;
        const int64_t need = m->eng->slot(m->slot).plan.n * int64_t(m->nvar) * CELLS;
        if (!u_out || capacity_doubles < need) return fail(m, AGILE_EINVAL, "output too small");
        MeshParams hp;
        if ((e = mesh_flags(m, hp))) return e;
        std::string s;
        int rc = m->eng->read_state(m->slot, u_out, out_on_device, s);
        return rc ? fail(m, rc, s) : AGILE_OK;
    });
}

int agile_read_ghosts(agile_mesh *m, double *g_out, int64_t capacity_doubles, int out_on_device) {
    return guarded(m, [&]() -> int {
        int e = usable(m);
        if (e) return e;
        if (m->te != 1) return fail(m, AGILE_EINVAL, "face ghosts are read per 16^3 block: block_n must be 16");
        const int64_t need = m->eng->slot(m->slot).plan.n * 6 * int64_t(m->nvar) * SLAB;
        if (!g_out || capacity_doubles < need) return fail(m, AGILE_EINVAL, "output too small");
        std::string s;
        int rc = m->eng->read_ghosts(m->slot, g_out, out_on_device, s);
        return rc ? fail(m, rc, s) : AGILE_OK;
    });
}

int agile_profile(agile_mesh *m, int kinds) {
    return guarded(m, [&]() -> int {
        int e = usable(m);
        if (e) return e;
        if (kinds < 0 || kinds > (AGILE_PROFILE_ALL | AGILE_PROFILE_KEEP)) return AGILE_EINVAL;
        std::string s;
        int rc = m->eng->profile(kinds, s);
        return rc ? fail(m, rc, s) : AGILE_OK;
    });
}

int agile_profile_read(agile_mesh *m, int kind, double *ms_total, int64_t *launches) {
    return guarded(m, [&]() -> int {
        int e = usable(m);
        if (e) return e;
        if (kind < 0 || kind > 3) return AGILE_EINVAL;
        double ms = 0;
        int64_t n = 0;
        std::string s;
        int rc = m->eng->profile_read(kind, ms, n, s);
        if (rc) return fail(m, rc, s);
        if (ms_total) *ms_total = ms;
        if (launches) *launches = n;
        return AGILE_OK;
    });
}

int agile_mesh_info(const agile_mesh *m, int64_t *nblocks, int *nvar) {
    return guarded(static_cast<agile_mesh *>(nullptr), [&]() -> int {
        if (!m) return AGILE_EINVAL;
        if (nblocks) *nblocks = m->eng ? int64_t(m->blocks.size()) : 0;
        if (nvar) *nvar = m->nvar;
        return AGILE_OK;
    });
}

void agile_mesh_destroy(agile_mesh *m) {
    if (!m) return;
    if (m->eng) (void)hipStreamSynchronize(m->eng->stream());
    delete m;
}

// ---------------------------------------------------------------------------
// batched serving

const char *agile_batch_last_error(const agile_batch *b) { return b ? b->msg.c_str() : ""; }

int agile_batch_create(const agile_batch_config *cfg, agile_batch **out) {
    return guarded(static_cast<agile_mesh *>(nullptr), [&]() -> int {
        if (!cfg || !out) return AGILE_EINVAL;
        // the pool holds 5-variable blocks: Euler (any solver) or SRHD (LF)
        const bool euler = cfg->physics == AGILE_EULER &&
                           (cfg->riemann == AGILE_HLL || cfg->riemann == AGILE_HLLC || cfg->riemann == AGILE_LF);
        const bool srhd = cfg->physics == AGILE_SRHD && cfg->riemann == AGILE_LF;
        if (!(euler || srhd) || (cfg->precision != AGILE_FP64 && cfg->precision != AGILE_FP32_FLUX) ||
            cfg->max_meshes < 1 || cfg->max_active_blocks < 0)
            return AGILE_EINVAL;
        if (cfg->dev_pool && cfg->dev_pool_bytes == 0) return AGILE_EINVAL;
        const int64_t budget = cfg->dev_pool ? int64_t(cfg->dev_pool_bytes)
                                             : (cfg->budget_bytes > 0 ? cfg->budget_bytes : (int64_t(16) << 30));
        // pool: blocks plus 1.5 ghost slabs and 1.5 flux registers per block (a
        // nested 2:1 mesh needs up to ~1.4 of each per block, a uniform one
        // none): the largest block count whose engine fits in the budget
        EngineConfig ec;
        ec.physics = cfg->physics;
        ec.riemann = cfg->riemann;
        ec.precision = cfg->precision;
        ec.stream = reinterpret_cast<hipStream_t>(cfg->stream);
        ec.cap_meshes = cfg->max_meshes;
        ec.pool = cfg->dev_pool;
        ec.pool_bytes = cfg->dev_pool_bytes;
        auto size_for = [&](int64_t cap) {
            ec.cap_blocks = int(cap);
            ec.cap_halo = int(cap + cap / 2);
            ec.cap_freg = int(cap + cap / 2);
            return int64_t(engine_device_bytes(ec));
        };
        int64_t lo = 0, hi = int64_t(1) << 30;
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) / 2;
            (size_for(mid) <= budget ? lo : hi) = mid;
        }
        if (lo < 1) return AGILE_ENOMEM;
        (void)size_for(lo);
        std::unique_ptr<agile_batch> b(new (std::nothrow) agile_batch());
        if (!b) return AGILE_ENOMEM;
        b->cfg = *cfg;
        b->eng.reset(new (std::nothrow) Engine());
        std::string e;
        int rc = b->eng ? b->eng->init(ec, e) : AGILE_ENOMEM;
        if (rc) return rc;
        b->eng->use_graph = cfg->use_graph != 0;
        *out = b.release();
        return AGILE_OK;
    });
}

int agile_batch_capacity(const agile_batch *b, int64_t *cap_blocks, int64_t *free_blocks) {
    return guarded(static_cast<agile_mesh *>(nullptr), [&]() -> int {
        if (!b) return AGILE_EINVAL;
        if (cap_blocks) *cap_blocks = b->eng->cap_blocks();
        if (free_blocks) *free_blocks = b->eng->free_blocks();
        return AGILE_OK;
    });
}

int agile_batch_submit(agile_batch *b, const agile_config *mesh_cfg, int64_t nblocks, const agile_block_desc *blocks,
                       const double *u, int u_on_device, int64_t nsteps, uint64_t tag) {
    return guarded(b, [&]() -> int {
        if (!b) return AGILE_EINVAL;
        if (b->err != AGILE_OK) return AGILE_ESTATE;
        if (check_config(mesh_cfg) != AGILE_OK || !u || nsteps < 1 || mesh_cfg->dev_pool || mesh_cfg->block_n != BN)
            return AGILE_EINVAL;
        // every request runs the batch's scheme
        if (mesh_cfg->physics != b->cfg.physics || mesh_cfg->riemann != b->cfg.riemann ||
            mesh_cfg->precision != b->cfg.precision || mesh_cfg->limiter != AGILE_MINMOD || mesh_cfg->rk_stages == 3)
            return AGILE_EINVAL;
        if (b->resident.count(tag)) return AGILE_EINVAL;
        for (const auto &r : b->queue)
            if (r.tag == tag) return AGILE_EINVAL;
        agile_batch::Request r;
        r.cfg = *mesh_cfg;
        std::string e;
        if (b->eng->plan(*mesh_cfg, nblocks, blocks, r.plan, e) != AGILE_OK) return AGILE_EINVAL;
        // can never be admitted
        if (r.plan.n > b->eng->cap_blocks() || r.plan.nhalo > b->eng->cap_halo() || r.plan.nfreg > b->eng->cap_freg())
            return AGILE_ENOMEM;
        if (u_on_device) r.dev = u;
        else r.u.assign(u, u + size_t(nblocks) * 5 * CELLS);
        r.blocks.assign(blocks, blocks + nblocks);
        r.steps = nsteps;
        r.tag = tag;
        b->queue.push_back(std::move(r));
        return AGILE_OK;
    });
}

int agile_batch_tick(agile_batch *b, agile_tick_info *info) {
    return guarded(b, [&]() -> int {
        if (!b) return AGILE_EINVAL;
        if (b->err != AGILE_OK) return AGILE_ESTATE;
        Engine &E = *b->eng;
        agile_tick_info ti{};
        std::string e;
        const double build0 = E.build_ms;
        const int64_t graphs0 = E.graph_builds;
        const auto t_admit = std::chrono::steady_clock::now();
        // admission: first come, first served, while the head of the queue fits
        // in memory and in the step-latency budget
        int64_t running = 0;
        for (const auto &kv : b->resident)
            if (E.slot(kv.second).active) running += E.slot(kv.second).plan.n;
        const int64_t budget = b->cfg.max_active_blocks;
        while (!b->queue.empty() && E.fits(b->queue.front().plan) &&
               (budget <= 0 || running == 0 || running + b->queue.front().plan.n <= budget)) {
            running += b->queue.front().plan.n;
            agile_batch::Request &r = b->queue.front();
            int slot = -1;
            const MeshParams *carry = r.has_carry ? &r.carry : nullptr;
            int rc = r.dev ? E.add(r.cfg, std::move(r.plan), r.dev, 1, r.steps, r.tag, &slot, e, carry)
                           : E.add(r.cfg, std::move(r.plan), r.u.data(), 0, r.steps, r.tag, &slot, e, carry);
            if (rc) return fail(b, rc, e);
            E.set_progress(slot, r.done);
            b->resident[r.tag] = slot;
            b->res_blocks[r.tag] = std::move(r.blocks);
            b->queue.pop_front();
            ti.admitted++;
        }
        ti.admit_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_admit).count();
        int64_t act_blocks = 0, act = 0;
        for (const auto &kv : b->resident) {
            const MeshSlot &S = E.slot(kv.second);
            if (S.active) {
                act++;
                act_blocks += S.plan.n;
            }
        }
        // stage shape per size class of the active set (tuned once per class)
        if (b->cfg.autotune && act_blocks > 0) {
            // power-of-two size classes; from 4096 blocks on the tuner's sample is
            // the same size, so those classes share one result
            int cls = 0;
            while ((int64_t(1) << (cls + 1)) <= act_blocks && cls < 12) cls++;
            auto it = b->tuned.find(cls);
            if (it == b->tuned.end()) {
                int rc = E.tune(e);
                if (rc) return fail(b, rc, e);
                b->tuned[cls] = {E.kslab, E.xcd, E.kslab_last, E.xcd_last};
            } else if (E.kslab != it->second[0] || E.xcd != it->second[1] || E.kslab_last != it->second[2] ||
                       E.xcd_last != it->second[3]) {
                E.kslab = it->second[0];
                E.xcd = it->second[1];
                E.kslab_last = it->second[2];
                E.xcd_last = it->second[3];
                for (const auto &kv : b->resident)   // the captured graph holds the old shape
                    if (E.slot(kv.second).active) {
                        E.set_active(kv.second, false);
                        E.set_active(kv.second, true);
                        break;
                    }
            }
        }
        if (act > 0) {
            int rc = E.step_cfl(1, e);
            if (rc) return fail(b, rc, e);
            if (hipStreamSynchronize(E.stream()) != hipSuccess) return fail(b, AGILE_EDEVICE, "step failed");
        }
        for (const auto &kv : b->resident) {
            const MeshSlot &S = E.slot(kv.second);
            if (S.active && S.steps_target >= 0 && S.steps_done >= S.steps_target) {
                E.set_active(kv.second, false);
                ti.finished++;
            }
        }
        ti.queued = int64_t(b->queue.size());
        ti.resident = int64_t(b->resident.size());
        ti.active = act;
        ti.active_blocks = act_blocks;
        ti.free_blocks = E.free_blocks();
        ti.build_ms = E.build_ms - build0;
        ti.graph_builds = E.graph_builds - graphs0;
        if (info) *info = ti;
        return AGILE_OK;
    });
}

int agile_batch_status(agile_batch *b, uint64_t tag, int *state, int64_t *steps_done) {
    return guarded(b, [&]() -> int {
        if (!b || !state) return AGILE_EINVAL;
        *state = AGILE_REQ_UNKNOWN;
        if (steps_done) *steps_done = 0;
        for (const auto &r : b->queue)
            if (r.tag == tag) {
                *state = AGILE_REQ_QUEUED;
                if (steps_done) *steps_done = r.done;
            }
        auto it = b->resident.find(tag);
        if (it != b->resident.end()) {
            const MeshSlot &S = b->eng->slot(it->second);
            *state = S.active ? AGILE_REQ_RUNNING : AGILE_REQ_FINISHED;
            if (steps_done) *steps_done = S.steps_done;
        }
        return AGILE_OK;
    });
}

int agile_batch_result(agile_batch *b, uint64_t tag, double *u_out, int64_t capacity_doubles, int out_on_device,
                       int64_t *steps_done, double *t_reached) {
    return guarded(b, [&]() -> int {
        if (!b) return AGILE_EINVAL;
        if (b->err != AGILE_OK) return AGILE_ESTATE;
        auto it = b->resident.find(tag);
        if (it == b->resident.end()) return AGILE_EINVAL;
        Engine &E = *b->eng;
        const int slot = it->second;
        const MeshSlot &S = E.slot(slot);
        if (S.active) return AGILE_ESTATE;   // still running
        const int64_t need = S.plan.n * 5 * int64_t(CELLS);
        if (!u_out || capacity_doubles < need) return AGILE_EINVAL;
        std::string e;
        MeshParams hp;
        int rc = E.read_params(slot, hp, e);
        if (rc) return fail(b, rc, e);
        rc = E.read_state(slot, u_out, out_on_device, e);
        if (rc) return fail(b, rc, e);
        if (out_on_device && hipStreamSynchronize(E.stream()) != hipSuccess) return fail(b, AGILE_EDEVICE, "readback");
        if (steps_done) *steps_done = S.steps_done;
        if (t_reached) *t_reached = hp.t;
        E.remove(slot);
        b->resident.erase(it);
        b->res_blocks.erase(tag);
        return (hp.flags & 1) ? AGILE_ENONPHYSICAL : AGILE_OK;
    });
}

int agile_batch_cancel(agile_batch *b, uint64_t tag) {
    return guarded(b, [&]() -> int {
        if (!b) return AGILE_EINVAL;
        for (auto q = b->queue.begin(); q != b->queue.end(); ++q)
            if (q->tag == tag) {
                b->queue.erase(q);
                return AGILE_OK;
            }
        auto it = b->resident.find(tag);
        if (it == b->resident.end()) return AGILE_EINVAL;
        b->eng->remove(it->second);
        b->resident.erase(it);
        b->res_blocks.erase(tag);
        return AGILE_OK;
    });
}

void agile_batch_destroy(agile_batch *b) {
    if (!b) return;
    if (b->eng) (void)hipStreamSynchronize(b->eng->stream());
    delete b;
}

} // extern "C"

// ---------------------------------------------------------------------------
// regrid

namespace {

int check_regrid_params(const agile_config &cfg, const agile_regrid_params *p, int nvar, std::string &msg) {
    if (!p) {
        msg = "null regrid parameters";
        return AGILE_EINVAL;
    }
    if (p->variable < 0 || p->variable >= nvar || !(p->eps > 0.0) || p->max_level < 1 ||
        p->max_level > cfg.max_level || !(p->refine == p->refine) || !(p->coarsen == p->coarsen)) {
        msg = "regrid parameters: variable, eps > 0, 1 <= max_level <= cfg.max_level, thresholds not NaN";
        return AGILE_EINVAL;
    }
    return AGILE_OK;
}

} // namespace

// Loehner estimate per block of a mesh (caller order): the maximum over the
// block's tiles.
int block_error(agile_mesh *m, int variable, double eps, double *out, std::string &e) {
    if (m->te == 1) return m->eng->lohner(m->slot, variable, eps, out, e);
    const size_t t3 = size_t(m->te) * m->te * m->te, n = m->blocks.size();
    std::vector<double> t(n * t3);
    const int rc = m->eng->lohner(m->slot, variable, eps, t.data(), e);
    if (rc) return rc;
    for (size_t q = 0; q < n; ++q) out[q] = *std::max_element(t.begin() + q * t3, t.begin() + (q + 1) * t3);
    return AGILE_OK;
}

int agile_mesh_error(agile_mesh *m, int variable, double eps, double *out_host) {
    return guarded(m, [&]() -> int {
        if (!m) return AGILE_EINVAL;
        if (m->err != AGILE_OK) return AGILE_ESTATE;
        if (!m->eng) return fail(m, AGILE_ESTATE, "no blocks set");
        if (!out_host) return fail(m, AGILE_EINVAL, "null output");
        std::string e;
        const int rc = block_error(m, variable, eps, out_host, e);
        return rc ? fail(m, rc, e) : AGILE_OK;
    });
}

int agile_regrid_decide(const agile_config *cfg, int64_t nblocks, const agile_block_desc *blocks, const double *err,
                        const agile_regrid_params *p, int64_t capacity, agile_block_desc *out, int64_t *n_out,
                        agile_regrid_stats *stats) {
    return guarded(static_cast<agile_mesh *>(nullptr), [&]() -> int {
        if (!cfg || !blocks || !err || !n_out || check_config(cfg) != AGILE_OK) return AGILE_EINVAL;
        std::string msg;
        const int nvar = cfg->physics == AGILE_MHD_GLM ? 9 : 5;
        if (check_regrid_params(*cfg, p, nvar, msg)) return AGILE_EINVAL;
        Plan P;
        PlanInput in{{cfg->base_blocks[0], cfg->base_blocks[1], cfg->base_blocks[2]}, cfg->max_level};
        if (build_plan(in, nblocks, blocks, P) != AGILE_OK) return AGILE_EINVAL;   // the old mesh must be valid
        std::vector<agile_block_desc> nb;
        std::vector<RegridSource> src;
        int64_t r = 0, c = 0;
        if (regrid_decide(in, nblocks, blocks, err, p->max_level, p->refine, p->coarsen, nb, src, r, c, msg) != AGILE_OK)
            return AGILE_EINVAL;
        *n_out = int64_t(nb.size());
        if (stats) *stats = agile_regrid_stats{nblocks, int64_t(nb.size()), r, c};
        if (int64_t(nb.size()) > capacity || (!out && !nb.empty())) return AGILE_EINVAL;
        std::copy(nb.begin(), nb.end(), out);
        return AGILE_OK;
    });
}

// Regrid of a single mesh (agile_mesh_regrid).  With `tasks` (device room
// for tasks_cap remap task records) nothing is allocated on the device: the
// new mesh must fit in the mesh's device pool and have at most tasks_cap
// blocks, else AGILE_ENOMEM / AGILE_EINVAL is returned with the mesh
// unchanged (not a sticky error).
int mesh_regrid(agile_mesh *m, const agile_regrid_params *p, agile_regrid_stats *stats, RemapTask *tasks,
                int64_t tasks_cap) {
    if (!m) return AGILE_EINVAL;
    if (m->err != AGILE_OK) return AGILE_ESTATE;
    if (!m->eng) return fail(m, AGILE_ESTATE, "no blocks set");
    std::string e;
    if (check_regrid_params(m->cfg, p, m->nvar, e)) return fail(m, AGILE_EINVAL, e);
    const int64_t n = int64_t(m->blocks.size());
    std::vector<double> err(static_cast<size_t>(n));
    int rc = block_error(m, p->variable, p->eps, err.data(), e);
    if (rc) return fail(m, rc, e);
    PlanInput in{{m->cfg.base_blocks[0], m->cfg.base_blocks[1], m->cfg.base_blocks[2]}, m->cfg.max_level};
    std::vector<agile_block_desc> nb;
    std::vector<RegridSource> src;
    int64_t r = 0, c = 0;
    rc = regrid_decide(in, n, m->blocks.data(), err.data(), p->max_level, p->refine, p->coarsen, nb, src, r, c, e);
    if (rc) return fail(m, rc, e);
    Plan P;
    if (plan_blocks(m->cfg, int64_t(nb.size()), nb.data(), P) != AGILE_OK)
        return fail(m, AGILE_EINVAL, "regrid: " + P.error);
    if (stats) *stats = agile_regrid_stats{n, int64_t(nb.size()), r, c};
    if (m->te != 1) {   // the decision is per block, the transfer per tile
        const std::vector<agile_block_desc> ot = expand_tiles(n, m->blocks.data(), m->te);
        const std::vector<agile_block_desc> nt = expand_tiles(int64_t(nb.size()), nb.data(), m->te);
        if (regrid_sources(ot, nt, src, e) != AGILE_OK) return fail(m, AGILE_EINVAL, e);
    }
    // the new state is staged in the stage buffer when the new mesh fits in
    // this pool; a mesh that outgrows it gets a new pool (not with a caller's
    // pool, nor without allocation)
    const bool in_place = m->eng->fits_replacing(m->slot, P);
    if (tasks && int64_t(src.size()) > tasks_cap)
        return refuse(m, AGILE_EINVAL, "regrid: " + std::to_string(src.size()) + " new 16^3 tiles exceed the limit of " +
                                           std::to_string(tasks_cap) + " of a regrid without allocation");
    if (!in_place && (tasks || m->cfg.dev_pool))
        return refuse(m, AGILE_ENOMEM, "regrid: the new mesh (" + std::to_string(nb.size()) +
                                           " blocks) does not fit in the mesh's device pool");
    double *d_new = in_place ? m->eng->stage_buffer(int64_t(src.size())) : nullptr;
    if (!d_new) {
        const size_t per = size_t(m->nvar) * CELLS;
        if (hipMalloc(&d_new, std::max<size_t>(1, src.size()) * per * sizeof(double)) != hipSuccess)
            return fail(m, AGILE_ENOMEM, "regrid: device buffer for the new state");
    }
    const bool own_new = !in_place;
    auto release = [&]() {
        if (own_new) (void)hipFree(d_new);
    };
    rc = m->eng->remap(m->slot, src, d_new, e, tasks);
    if (rc) {
        release();
        return fail(m, rc, e);
    }
    // simulated time, last dt and the non-physical flag carry over
    MeshParams carry{};
    rc = m->eng->read_params(m->slot, carry, e);
    if (rc) {
        release();
        return fail(m, rc, e);
    }
    // the old mesh is no longer read
    (void)m->eng->remove(m->slot);
    m->slot = -1;
    if (in_place) {
        int slot = -1;
        rc = m->eng->add(m->tcfg, std::move(P), d_new, 1, -1, 0, &slot, e, &carry, 1, m->te);
        if (rc == AGILE_OK) {
            m->slot = slot;
            m->blocks = nb;
        } else {
            rc = fail(m, rc, e);
        }
    } else {
        rc = new_engine(m, std::move(P), int64_t(nb.size()), nb.data(), d_new, 1, 1.5, &carry, 1);
    }
    if (m->eng) (void)hipStreamSynchronize(m->eng->stream());
    release();
    return rc;
}

int agile_mesh_regrid(agile_mesh *m, const agile_regrid_params *p, agile_regrid_stats *stats) {
    return guarded(m, [&]() -> int { return mesh_regrid(m, p, stats, nullptr, 0); });
}

int agile_copy_probe(void *dst, const void *src, size_t bytes, void *stream) {
    return guarded(static_cast<agile_mesh *>(nullptr), [&]() -> int {
        if ((!dst || !src) && bytes) return AGILE_EINVAL;
        if (bytes % 16 || reinterpret_cast<uintptr_t>(dst) % 16 || reinterpret_cast<uintptr_t>(src) % 16)
            return AGILE_EINVAL;
        return launch_stream_copy(src, dst, bytes, reinterpret_cast<hipStream_t>(stream)) == hipSuccess
                   ? AGILE_OK
                   : AGILE_EDEVICE;
    });
}

int agile_mesh_regrid_noalloc(agile_mesh *m, const agile_regrid_params *p, agile_regrid_stats *stats) {
    return guarded(m, [&]() -> int {
        if (!m) return AGILE_EINVAL;
        if (m->err != AGILE_OK) return AGILE_ESTATE;
        if (!m->eng) return fail(m, AGILE_ESTATE, "no blocks set");
        int dev = -1;
        if (hipGetDevice(&dev) != hipSuccess || dev != m->device)
            return refuse(m, AGILE_EINVAL, "regrid without allocation: the mesh's device must be current");
        std::string e;
        RemapTask *tasks = noalloc_scratch(dev, e);
        if (!tasks) return fail(m, AGILE_EDEVICE, e);
        return mesh_regrid(m, p, stats, tasks, AGILE_NOALLOC_MAX_BLOCKS);
    });
}

int agile_batch_regrid(agile_batch *b, uint64_t tag, const agile_regrid_params *p, agile_regrid_stats *stats) {
    return guarded(b, [&]() -> int {
        if (!b) return AGILE_EINVAL;
        if (b->err != AGILE_OK) return AGILE_ESTATE;
        auto it = b->resident.find(tag);
        if (it == b->resident.end()) return AGILE_EINVAL;     // unknown, queued or collected
        Engine &E = *b->eng;
        const int slot = it->second;
        if (!E.slot(slot).active) return AGILE_EINVAL;        // finished: nothing left to step
        const agile_config cfg = E.slot(slot).cfg;
        const int64_t target = E.slot(slot).steps_target, done = E.slot(slot).steps_done;
        std::string e;
        if (check_regrid_params(cfg, p, 5, e)) return AGILE_EINVAL;
        const std::vector<agile_block_desc> &old = b->res_blocks[tag];
        const int64_t n = int64_t(old.size());
        std::vector<double> err(static_cast<size_t>(n));
        int rc = E.lohner(slot, p->variable, p->eps, err.data(), e);
        if (rc) return fail(b, rc, e);
        PlanInput in{{cfg.base_blocks[0], cfg.base_blocks[1], cfg.base_blocks[2]}, cfg.max_level};
        std::vector<agile_block_desc> nb;
        std::vector<RegridSource> src;
        int64_t r = 0, c = 0;
        rc = regrid_decide(in, n, old.data(), err.data(), p->max_level, p->refine, p->coarsen, nb, src, r, c, e);
        if (rc) return AGILE_EINVAL;
        if (stats) *stats = agile_regrid_stats{n, int64_t(nb.size()), r, c};
        Plan P;
        if (E.plan(cfg, int64_t(nb.size()), nb.data(), P, e) != AGILE_OK) return AGILE_EINVAL;
        // a mesh larger than the whole pool could never be admitted again
        if (P.n > E.cap_blocks() || P.nhalo > E.cap_halo() || P.nfreg > E.cap_freg()) return AGILE_ENOMEM;
        MeshParams carry{};
        if ((rc = E.read_params(slot, carry, e))) return fail(b, rc, e);
        const size_t per = size_t(5) * CELLS;
        // in place when the new mesh fits beside the others (state staged in
        // the stage buffer, free between ticks); else it leaves the pool and
        // rejoins the queue at its head with its state on the host
        const bool in_place = E.fits_replacing(slot, P);
        double *d_new = in_place ? E.stage_buffer(P.n) : nullptr;
        if (!d_new && hipMalloc(&d_new, std::max<size_t>(1, nb.size()) * per * sizeof(double)) != hipSuccess)
            return fail(b, AGILE_ENOMEM, "batch regrid: device buffer for the new state");
        auto release = [&]() {
            if (!in_place) (void)hipFree(d_new);
        };
        if ((rc = E.remap(slot, src, d_new, e))) {
            release();
            return fail(b, rc, e);
        }
        agile_batch::Request q;
        if (!in_place) {
            q.u.resize(nb.size() * per);
            const hipError_t he = hipMemcpy(q.u.data(), d_new, q.u.size() * sizeof(double), hipMemcpyDeviceToHost);
            release();
            if (he != hipSuccess) return fail(b, AGILE_EDEVICE, "batch regrid: state copy");
        }
        E.remove(slot);
        b->resident.erase(it);
        if (in_place) {
            int ns = -1;
            rc = E.add(cfg, std::move(P), d_new, 1, target, tag, &ns, e, &carry);
            if (rc) return fail(b, rc, e);
            E.set_progress(ns, done);
            b->resident[tag] = ns;
            b->res_blocks[tag] = std::move(nb);
            return AGILE_OK;
        }
        b->res_blocks.erase(tag);
        q.cfg = cfg;
        q.plan = std::move(P);
        q.blocks = std::move(nb);
        q.steps = target;
        q.tag = tag;
        q.done = done;
        q.has_carry = true;
        q.carry = carry;
        b->queue.push_front(std::move(q));
        return AGILE_OK;
    });
}

int agile_batch_blocks(agile_batch *b, uint64_t tag, int64_t capacity, agile_block_desc *out, int64_t *n) {
    return guarded(b, [&]() -> int {
        if (!b || !n) return AGILE_EINVAL;
        const std::vector<agile_block_desc> *bl = nullptr;
        auto it = b->res_blocks.find(tag);
        if (it != b->res_blocks.end()) bl = &it->second;
        for (const auto &r : b->queue)
            if (r.tag == tag) bl = &r.blocks;
        if (!bl) return AGILE_EINVAL;
        *n = int64_t(bl->size());
        if (*n > capacity || (!out && *n > 0)) return AGILE_EINVAL;
        std::copy(bl->begin(), bl->end(), out);
        return AGILE_OK;
    });
}

int agile_mesh_blocks(const agile_mesh *m, int64_t capacity, agile_block_desc *out, int64_t *n) {
    return guarded(static_cast<agile_mesh *>(nullptr), [&]() -> int {
        if (!m || !n) return AGILE_EINVAL;
        *n = int64_t(m->blocks.size());
        if (*n > capacity || (!out && *n > 0)) return AGILE_EINVAL;
        std::copy(m->blocks.begin(), m->blocks.end(), out);
        return AGILE_OK;
    });
}
