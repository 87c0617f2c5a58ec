"""Regrid decision of the oracle: which leaves to refine or coarsen, with the
2:1 balance across faces kept.

TEST INFRASTRUCTURE ONLY (like the rest of oracle/): plain Python loops over
the block list, written from the description of the regrid step (the "AMR
error estimator" and "AMR Coarsen Refine" nodes of the flow charts, Fig. 1
and Fig. 2).

Readings (the paper gives no rule):
  - a leaf is flagged for refinement when its estimator exceeds `refine`
    and its level is below `max_level`;
  - a complete octet of sibling leaves (level >= 2) is flagged for
    coarsening when every one of the eight is below `coarsen` and none is
    flagged for refinement;
  - balance: a leaf that would end up with a face neighbour two levels finer
    is refined too (repeated until nothing changes); then an octet whose
    parent would have a face neighbour two levels finer is not coarsened
    (repeated until nothing changes);
  - one level of change per leaf and regrid; periodic domain;
  - the new list is sorted by (level, bx, by, bz).
"""
from __future__ import annotations


def _leaf_at(leaves, base, l, c):
    """The leaf (level, bx, by, bz) that covers level-l block c (periodic), or
    None when finer leaves cover it."""
    n = [b << (l - 1) for b in base]
    c = [c[d] % n[d] for d in range(3)]
    for L in range(l, 0, -1):
        key = (L, c[0] >> (l - L), c[1] >> (l - L), c[2] >> (l - L))
        if key in leaves:
            return key
    return None


def _face_neighbours(leaves, base, leaf):
    """Levels of the leaves that touch a face of `leaf` (any level)."""
    l, x, y, z = leaf
    out = []
    for d in range(3):
        for s in (-1, 1):
            c = [x, y, z]
            c[d] += s
            hit = _leaf_at(leaves, base, l, c)
            if hit is not None:
                out.append(hit[0])
                continue
            # covered by finer leaves: the children of that block touching the face
            stack = [(l, c)]
            while stack:
                L, cc = stack.pop()
                for dz in range(2):
                    for dy in range(2):
                        for dx in range(2):
                            ch = [2 * cc[0] + dx, 2 * cc[1] + dy, 2 * cc[2] + dz]
                            # keep the children on the side facing `leaf`
                            if ch[d] % 2 != (1 if s < 0 else 0):
                                continue
                            n = [b << L for b in base]
                            ch = [ch[e] % n[e] for e in range(3)]
                            key = (L + 1, *ch)
                            if key in leaves:
                                out.append(L + 1)
                            else:
                                stack.append((L + 1, ch))
    return out


def _build(leaves, refine, coarsen_parents):
    new = set(leaves)
    for (l, x, y, z) in refine:
        new.discard((l, x, y, z))
        for dz in range(2):
            for dy in range(2):
                for dx in range(2):
                    new.add((l + 1, 2 * x + dx, 2 * y + dy, 2 * z + dz))
    for (l, x, y, z) in coarsen_parents:
        for dz in range(2):
            for dy in range(2):
                for dx in range(2):
                    new.discard((l + 1, 2 * x + dx, 2 * y + dy, 2 * z + dz))
        new.add((l, x, y, z))
    return new


def decide(blocks, err, base, max_level, refine, coarsen):
    """blocks: (level, bx, by, bz) leaves; err: estimator per leaf.  Returns
    (new sorted leaf list, refined leaves, coarsened parents)."""
    leaves = {tuple(int(v) for v in b): float(e) for b, e in zip(blocks, err)}
    R = {b for b, e in leaves.items() if e > refine and b[0] < max_level}
    # refinement balance: a leaf next to a leaf being refined must not end up
    # two levels coarser than the new children
    changed = True
    while changed:
        changed = False
        for b in sorted(R):
            l = b[0]
            for d in range(3):
                for s in (-1, 1):
                    c = list(b[1:])
                    c[d] += s
                    hit = _leaf_at(leaves, base, l, c)
                    if hit is not None and hit[0] < l and hit not in R:
                        R.add(hit)
                        changed = True
    # coarsening candidates: complete octets of low-error leaves
    parents = {}
    for (l, x, y, z) in leaves:
        if l >= 2:
            parents.setdefault((l - 1, x >> 1, y >> 1, z >> 1), []).append((l, x, y, z))
    P = set()
    for p, kids in parents.items():
        if len(kids) == 8 and all(leaves[k] < coarsen and k not in R for k in kids):
            P.add(p)
    # coarsening balance
    changed = True
    while changed:
        changed = False
        new = _build(leaves, R, P)
        for p in sorted(P):
            if any(L > p[0] + 1 for L in _face_neighbours(new, base, p)):
                P.discard(p)
                changed = True
                break
    new = _build(leaves, R, P)
    return sorted(new), sorted(R), sorted(P)
