// regrid.cpp -- host side of a regrid: the refine / coarsen decision from the
// device error estimate and the data source of every new leaf (the "AMR
// Coarsen Refine" node of the flow charts, Fig. 1 and Fig. 2, which the paper
// keeps on the host with the tree).
#include <algorithm>
#include <array>
#include <unordered_map>
#include <unordered_set>

#include "mesh.hpp"

namespace agile {

namespace {

struct Key {
    int l;
    int64_t x, y, z;
};

inline uint64_t pack(int l, int64_t x, int64_t y, int64_t z) {
    return (uint64_t(l) << 60) | (uint64_t(x) << 40) | (uint64_t(y) << 20) | uint64_t(z);
}

inline int64_t wrapc(int64_t c, int64_t n) {
    const int64_t r = c % n;
    return r < 0 ? r + n : r;
}

} // namespace

int regrid_decide(const PlanInput &in, int64_t n, const agile_block_desc *blocks, const double *err, int max_level,
                  double refine, double coarsen, std::vector<agile_block_desc> &out, std::vector<RegridSource> &src,
                  int64_t &refined, int64_t &coarsened, std::string &error) {
    out.clear();
    src.clear();
    refined = coarsened = 0;
    if (max_level < 1 || max_level > in.max_level) {
        error = "regrid: maximum level outside [1, the mesh's maximum level]";
        return AGILE_EINVAL;
    }
    auto dims = [&](int l, int d) { return int64_t(in.base[d]) << (l - 1); };
    std::unordered_map<uint64_t, int> leaf;
    leaf.reserve(size_t(2 * n));
    for (int64_t q = 0; q < n; ++q) leaf[pack(blocks[q].level, blocks[q].idx[0], blocks[q].idx[1], blocks[q].idx[2])] = int(q);
    // old leaf covering level-l block c, or -1 when finer leaves cover it
    auto covering = [&](int l, int64_t c[3]) -> int {
        for (int L = l; L >= 1; --L) {
            auto it = leaf.find(pack(L, c[0] >> (l - L), c[1] >> (l - L), c[2] >> (l - L)));
            if (it != leaf.end()) return it->second;
        }
        return -1;
    };

    // refinement and its propagation to coarser face neighbours
    std::vector<char> R(size_t(n), 0);
    std::vector<int> work;
    for (int64_t q = 0; q < n; ++q)
        if (err[q] > refine && blocks[q].level < max_level) {
            R[q] = 1;
            work.push_back(int(q));
        }
    while (!work.empty()) {
        const int q = work.back();
        work.pop_back();
        const int l = blocks[q].level;
        for (int d = 0; d < 3; ++d)
            for (int s = -1; s <= 1; s += 2) {
                int64_t c[3] = {blocks[q].idx[0], blocks[q].idx[1], blocks[q].idx[2]};
                c[d] = wrapc(c[d] + s, dims(l, d));
                const int h = covering(l, c);
                if (h >= 0 && blocks[h].level < l && !R[h]) {
                    R[h] = 1;
                    work.push_back(h);
                }
            }
    }

    // coarsening candidates: complete octets of low-error leaves, none refined
    std::unordered_map<uint64_t, std::array<int, 8>> octets;
    for (int64_t q = 0; q < n; ++q) {
        const agile_block_desc &b = blocks[q];
        if (b.level < 2) continue;
        auto &o = octets.try_emplace(pack(b.level - 1, b.idx[0] >> 1, b.idx[1] >> 1, b.idx[2] >> 1),
                                     std::array<int, 8>{-1, -1, -1, -1, -1, -1, -1, -1}).first->second;
        o[(b.idx[0] & 1) + 2 * (b.idx[1] & 1) + 4 * (b.idx[2] & 1)] = int(q);
    }
    std::vector<std::pair<uint64_t, std::array<int, 8>>> P;
    for (auto &kv : octets) {
        bool ok = true;
        for (int k : kv.second) ok = ok && k >= 0 && err[k] < coarsen && !R[k];
        if (ok) P.push_back(kv);
    }

    // the new leaf set for the current choice of coarsened octets
    auto build = [&](std::unordered_set<uint64_t> &nl) {
        nl.clear();
        std::unordered_set<int> gone;
        for (auto &p : P)
            for (int k : p.second) gone.insert(k);
        for (int64_t q = 0; q < n; ++q) {
            const agile_block_desc &b = blocks[q];
            if (gone.count(int(q))) continue;
            if (R[q]) {
                for (int o = 0; o < 8; ++o)
                    nl.insert(pack(b.level + 1, 2 * b.idx[0] + (o & 1), 2 * b.idx[1] + ((o >> 1) & 1),
                                   2 * b.idx[2] + (o >> 2)));
            } else {
                nl.insert(pack(b.level, b.idx[0], b.idx[1], b.idx[2]));
            }
        }
        for (auto &p : P) nl.insert(p.first);
    };
    // coarsening balance: withdraw octets whose parent would touch a leaf two
    // levels finer, until none does (withdrawing only refines neighbourhoods)
    std::unordered_set<uint64_t> nl;
    for (bool changed = true; changed;) {
        changed = false;
        build(nl);
        std::vector<std::pair<uint64_t, std::array<int, 8>>> keep;
        for (auto &p : P) {
            const int lp = int(p.first >> 60);
            const int64_t px = int64_t((p.first >> 40) & 0xfffff), py = int64_t((p.first >> 20) & 0xfffff),
                          pz = int64_t(p.first & 0xfffff);
            bool bad = false;
            for (int d = 0; d < 3 && !bad; ++d)
                for (int s = -1; s <= 1 && !bad; s += 2) {
                    int64_t c[3] = {px, py, pz};
                    c[d] = wrapc(c[d] + s, dims(lp, d));
                    bool covered = false;
                    for (int L = lp; L >= 1 && !covered; --L)
                        covered = nl.count(pack(L, c[0] >> (lp - L), c[1] >> (lp - L), c[2] >> (lp - L))) != 0;
                    if (covered) continue;
                    // subdivided: its children facing the parent must be leaves
                    for (int o = 0; o < 8 && !bad; ++o) {
                        const int64_t ch[3] = {2 * c[0] + (o & 1), 2 * c[1] + ((o >> 1) & 1), 2 * c[2] + (o >> 2)};
                        if ((ch[d] & 1) != (s < 0 ? 1 : 0)) continue;
                        if (!nl.count(pack(lp + 1, ch[0], ch[1], ch[2]))) bad = true;
                    }
                }
            if (bad) changed = true;
            else keep.push_back(p);
        }
        P.swap(keep);
    }
    build(nl);

    // the new leaves, sorted, with their sources
    std::unordered_map<uint64_t, int> parent_of_octet;
    for (size_t i = 0; i < P.size(); ++i) parent_of_octet[P[i].first] = int(i);
    std::vector<Key> keys;
    keys.reserve(nl.size());
    for (uint64_t k : nl)
        keys.push_back({int(k >> 60), int64_t((k >> 40) & 0xfffff), int64_t((k >> 20) & 0xfffff), int64_t(k & 0xfffff)});
    std::sort(keys.begin(), keys.end(), [](const Key &a, const Key &b) {
        if (a.l != b.l) return a.l < b.l;
        if (a.x != b.x) return a.x < b.x;
        if (a.y != b.y) return a.y < b.y;
        return a.z < b.z;
    });
    out.resize(keys.size());
    src.resize(keys.size());
    for (size_t i = 0; i < keys.size(); ++i) {
        const Key &k = keys[i];
        out[i].level = k.l;
        out[i].idx[0] = int(k.x);
        out[i].idx[1] = int(k.y);
        out[i].idx[2] = int(k.z);
        RegridSource &S = src[i];
        auto it = leaf.find(pack(k.l, k.x, k.y, k.z));
        auto po = parent_of_octet.find(pack(k.l, k.x, k.y, k.z));
        if (po != parent_of_octet.end()) {
            S.kind = 2;
            for (int o = 0; o < 8; ++o) S.src[o] = P[po->second].second[o];
        } else if (it != leaf.end()) {
            S.kind = 0;
            S.src[0] = it->second;
        } else {
            auto pp = leaf.find(pack(k.l - 1, k.x >> 1, k.y >> 1, k.z >> 1));
            if (pp == leaf.end() || !R[pp->second]) {
                error = "regrid: internal inconsistency";
                return AGILE_EINVAL;
            }
            S.kind = 1;
            S.src[0] = pp->second;
            S.octant = int((k.x & 1) + 2 * (k.y & 1) + 4 * (k.z & 1));
        }
    }
    for (char r : R) refined += r;
    coarsened = int64_t(P.size());
    return AGILE_OK;
}

// Data sources of the blocks `nw` of a regridded mesh from the blocks `old`
// of the same domain, by position: a block that exists in both is copied, one
// whose parent block is old is that parent's child, one whose 8 children are
// old is their mean.  (The tiles of a regrid of larger blocks, where the
// decision was taken per block.)
int regrid_sources(const std::vector<agile_block_desc> &old, const std::vector<agile_block_desc> &nw,
                   std::vector<RegridSource> &src, std::string &error) {
    std::unordered_map<uint64_t, int> at;
    at.reserve(2 * old.size());
    for (size_t q = 0; q < old.size(); ++q)
        at[pack(old[q].level, old[q].idx[0], old[q].idx[1], old[q].idx[2])] = int(q);
    src.assign(nw.size(), RegridSource{});
    for (size_t q = 0; q < nw.size(); ++q) {
        const agile_block_desc &b = nw[q];
        RegridSource &r = src[q];
        auto it = at.find(pack(b.level, b.idx[0], b.idx[1], b.idx[2]));
        if (it != at.end()) {
            r.kind = 0;
            r.src[0] = it->second;
            continue;
        }
        if (b.level > 1) {
            it = at.find(pack(b.level - 1, b.idx[0] >> 1, b.idx[1] >> 1, b.idx[2] >> 1));
            if (it != at.end()) {
                r.kind = 1;
                r.octant = int((b.idx[0] & 1) + 2 * (b.idx[1] & 1) + 4 * (b.idx[2] & 1));
                r.src[0] = it->second;
                continue;
            }
        }
        r.kind = 2;
        for (int o = 0; o < 8; ++o) {
            it = at.find(pack(b.level + 1, 2 * int64_t(b.idx[0]) + (o & 1), 2 * int64_t(b.idx[1]) + ((o >> 1) & 1),
                              2 * int64_t(b.idx[2]) + (o >> 2)));
            if (it == at.end()) {
                error = "regrid: a new block has no source in the old mesh";
                return AGILE_EINVAL;
            }
            r.src[o] = it->second;
        }
    }
    return AGILE_OK;
}

} // namespace agile
