// mesh.cpp -- host-side mesh bookkeeping of the block-AMR update.
//
// The paper keeps grid connectivity and neighbour relations on the host and
// rebuilds them whenever the mesh changes (Sec. 2.1.2; the nbinfo structure
// of Sec. 2.1.3 with its same-level / finer / coarser neighbour types).  This
// file does the same for a static leaf set: it validates the block list
// (range, duplicates, overlap, tiling of the periodic domain, 2:1 balance
// across faces), orders blocks by level and Morton code (the space-filling
// curve of Sec. 2.1.3) and builds flat tables the kernels read:
//   - per block and face: same-level neighbour, or the ghost slab filled by
//     restriction (finer neighbours) / prolongation (coarser neighbour);
//   - restriction tasks, prolongation tasks grouped by level (a fine ghost is
//     prolonged from a coarse block whose own ghosts must be complete);
//   - flux registers and one flux-correction task per coarse block.
#include "mesh.hpp"

#include <algorithm>
#include <cstring>
#include <unordered_map>

namespace agile {

namespace {

inline uint64_t key_of(int level, int64_t x, int64_t y, int64_t z) {
    return (uint64_t(level) << 60) | (uint64_t(x) << 40) | (uint64_t(y) << 20) | uint64_t(z);
}

inline uint64_t spread3(uint64_t v) {
    // spread the low 21 bits of v to every third bit
    v &= 0x1fffff;
    v = (v | (v << 32)) & 0x1f00000000ffffULL;
    v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
    v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
    v = (v | (v << 2)) & 0x1249249249249249ULL;
    return v;
}

inline uint64_t morton(int64_t x, int64_t y, int64_t z) {
    return spread3(uint64_t(x)) | (spread3(uint64_t(y)) << 1) | (spread3(uint64_t(z)) << 2);
}

inline int64_t wrap(int64_t c, int64_t n) {
    int64_t r = c % n;
    return r < 0 ? r + n : r;
}

// lower / upper tangential axes of a face normal to d
inline int tan_a(int d) { return d == 0 ? 1 : 0; }
inline int tan_b(int d) { return d == 2 ? 1 : 2; }

} // namespace

int build_plan(const PlanInput &in, int64_t n, const agile_block_desc *blocks, Plan &P) {
    P = Plan();
    auto fail = [&](const std::string &msg) {
        P.error = msg;
        return AGILE_EINVAL;
    };
    if (n <= 0) return fail("nblocks must be positive");
    if (n > (int64_t(1) << 30)) return fail("too many blocks");
    if (!blocks) return fail("null block list");
    const int L = in.max_level;
    int64_t nbl[MAXLEV + 1][3];
    for (int l = 1; l <= L; ++l)
        for (int d = 0; d < 3; ++d) nbl[l][d] = int64_t(in.base[d]) << (l - 1);
    for (int d = 0; d < 3; ++d)
        if (nbl[L][d] >= (int64_t(1) << 20)) return fail("too many blocks per axis on the finest level");

    std::unordered_map<uint64_t, int> where;
    where.reserve(size_t(n) * 2);
    for (int64_t q = 0; q < n; ++q) {
        const agile_block_desc &b = blocks[q];
        if (b.level < 1 || b.level > L) return fail("block " + std::to_string(q) + ": level out of range");
        for (int d = 0; d < 3; ++d)
            if (b.idx[d] < 0 || b.idx[d] >= nbl[b.level][d])
                return fail("block " + std::to_string(q) + ": index out of range");
        uint64_t k = key_of(b.level, b.idx[0], b.idx[1], b.idx[2]);
        if (!where.emplace(k, int(q)).second) return fail("block " + std::to_string(q) + ": duplicate");
    }
    // overlap (a leaf inside another leaf) and tiling by volume
    unsigned __int128 vol = 0, dom = (unsigned __int128)in.base[0] * in.base[1] * in.base[2];
    for (int l = 1; l < L; ++l) dom *= 8;
    for (int64_t q = 0; q < n; ++q) {
        const agile_block_desc &b = blocks[q];
        for (int l = b.level - 1; l >= 1; --l) {
            int s = b.level - l;
            if (where.count(key_of(l, b.idx[0] >> s, b.idx[1] >> s, b.idx[2] >> s)))
                return fail("block " + std::to_string(q) + ": overlaps a coarser block");
        }
        vol += (unsigned __int128)1 << (3 * (L - b.level));
    }
    if (vol != dom) return fail("blocks do not tile the domain (gap)");

    // device order: level, then Morton code
    P.n = n;
    P.order.resize(n);
    for (int64_t q = 0; q < n; ++q) P.order[q] = int(q);
    std::vector<uint64_t> mk(n);
    for (int64_t q = 0; q < n; ++q) mk[q] = morton(blocks[q].idx[0], blocks[q].idx[1], blocks[q].idx[2]);
    std::stable_sort(P.order.begin(), P.order.end(), [&](int a, int b) {
        if (blocks[a].level != blocks[b].level) return blocks[a].level < blocks[b].level;
        return mk[a] < mk[b];
    });
    P.perm.resize(n);
    for (int64_t q = 0; q < n; ++q) P.perm[P.order[q]] = int(q);
    auto dev_of = [&](int level, int64_t x, int64_t y, int64_t z) -> int {
        auto it = where.find(key_of(level, x, y, z));
        return it == where.end() ? -1 : P.perm[it->second];
    };

    P.desc.assign(n, BlockDesc{});
    P.prolong.assign(L + 1, {});
    P.levels = 0;
    // fine flux register slot of (fine block, face) -> slot, filled while
    // scanning the fine side; used by the coarse side afterwards
    std::unordered_map<uint64_t, int> fine_reg;
    for (int64_t db = 0; db < n; ++db) {
        const agile_block_desc &b = blocks[P.order[db]];
        BlockDesc &D = P.desc[db];
        D.level = b.level;
        D.mesh = 0;
        D.cf_coarse = 0;
        P.levels = std::max(P.levels, b.level);
        for (int f = 0; f < 6; ++f) {
            D.freg[f] = -1;
            int d = f / 2, side = f % 2;
            int64_t c[3] = {b.idx[0], b.idx[1], b.idx[2]};
            c[d] = wrap(c[d] + (side ? 1 : -1), nbl[b.level][d]);
            int same = dev_of(b.level, c[0], c[1], c[2]);
            if (same >= 0) {
                D.nb[f] = same;
                continue;
            }
            if (b.level > 1) {
                int coarse = dev_of(b.level - 1, c[0] >> 1, c[1] >> 1, c[2] >> 1);
                if (coarse >= 0) {
                    // this block is the fine side: ghost slab prolonged from `coarse`
                    ProlongTask t{};
                    t.slot = P.nhalo++;
                    t.face = f;
                    t.block = int(db);
                    t.coarse = coarse;
                    t.ta = 8 * int(b.idx[tan_a(d)] & 1);
                    t.tb = 8 * int(b.idx[tan_b(d)] & 1);
                    D.nb[f] = -(t.slot + 1);
                    P.prolong[b.level].push_back(t);
                    D.freg[f] = P.nfreg++;
                    fine_reg[uint64_t(db) * 8 + f] = D.freg[f];
                    continue;
                }
            }
            // finer: the 4 children of the neighbour region adjacent to this face
            if (b.level + 1 > L) return fail("2:1 balance / tiling violated next to block " + std::to_string(P.order[db]));
            RestrictTask t{};
            t.face = f;
            t.block = int(db);
            int ta = tan_a(d), tb = tan_b(d);
            for (int qb = 0; qb < 2; ++qb)
                for (int qa = 0; qa < 2; ++qa) {
                    int64_t fc[3];
                    fc[d] = 2 * c[d] + (side ? 0 : 1);
                    fc[ta] = 2 * int64_t(b.idx[ta]) + qa;
                    fc[tb] = 2 * int64_t(b.idx[tb]) + qb;
                    int fine = dev_of(b.level + 1, fc[0], fc[1], fc[2]);
                    if (fine < 0)
                        return fail("2:1 balance violated across a face of block " + std::to_string(P.order[db]));
                    t.fine[qa + 2 * qb] = fine;
                }
            t.slot = P.nhalo++;
            D.nb[f] = -(t.slot + 1);
            D.cf_coarse |= 1 << f;
            D.freg[f] = P.nfreg++;
            P.restrict_tasks.push_back(t);
        }
    }
    // Level dependencies of the prolongation: a task reads the coarse block's
    // cells next to the face, their normal neighbours (one inside, one in the
    // restricted slab on the fine side) and, at the edge of its 8 x 8 parent
    // patch, one tangential face per tangential axis.  If such a face of the
    // coarse block is itself a prolonged slab (coarser neighbour), the level
    // must wait for the level below; otherwise levels can share one launch.
    P.prolong_dep.assign(L + 1, 0);
    for (int l = 0; l <= L; ++l)
        for (const ProlongTask &t : P.prolong[l]) {
            const BlockDesc &C = P.desc[t.coarse];
            const int d = t.face / 2;
            const int fa = 2 * tan_a(d) + (t.ta == 8), fb = 2 * tan_b(d) + (t.tb == 8);
            for (int f : {fa, fb})
                if (C.nb[f] < 0 && !((C.cf_coarse >> f) & 1)) P.prolong_dep[l] = 1;
        }
    // flux-correction tasks, one per coarse block with coarse-fine faces
    for (const RestrictTask &t : P.restrict_tasks) {
        if (P.reflux.empty() || P.reflux.back().block != t.block) {
            RefluxTask r{};
            r.block = t.block;
            r.level = P.desc[t.block].level;
            r.nface = 0;
            P.reflux.push_back(r);
        }
        RefluxTask &r = P.reflux.back();
        int f = t.face;
        r.face[r.nface] = f;
        r.cslot[r.nface] = P.desc[t.block].freg[f];
        for (int q = 0; q < 4; ++q) {
            auto it = fine_reg.find(uint64_t(t.fine[q]) * 8 + (f ^ 1));
            if (it == fine_reg.end()) return fail("internal: missing fine flux register");
            r.fslot[r.nface][q] = it->second;
        }
        r.nface++;
    }
    return AGILE_OK;
}

size_t plan_device_bytes(const Plan &P, int nvar) {
    size_t b = 0;
    b += 2 * size_t(P.n) * nvar * CELLS * sizeof(double);      // U[2]
    b += 2 * size_t(P.n) * nvar * XE_CELLS * sizeof(double);   // XE[2]
    b += size_t(P.nhalo) * nvar * SLAB * sizeof(double);       // ghost slabs
    b += size_t(P.nfreg) * nvar * REG * sizeof(double);        // flux registers
    b += size_t(P.n) * (sizeof(BlockDesc) + sizeof(unsigned long long));
    size_t np = 0;
    for (const auto &v : P.prolong) np += v.size();
    b += P.restrict_tasks.size() * sizeof(RestrictTask) + np * sizeof(ProlongTask) +
         P.reflux.size() * sizeof(RefluxTask) + sizeof(MeshParams) + 2 * size_t(P.n) * sizeof(int);
    return b;
}

} // namespace agile
