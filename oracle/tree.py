"""Cluster tree, block cluster tree and translation classes (oracle; test infrastructure only).

Paper: Sec. 3.2 "Cluster Tree" and Alg. ConstructClusterTree (appendix);
Sec. 3.3 "Block Cluster Tree", the admissibility condition (eq. "admissible")
and Alg. ConstructBlockClusterTree; App. "Additional Definitions" (distance and
diameter of hypercubes); Sec. 5.2 "Translation Invariance".

Readings taken where the paper is silent or garbled:
* Alg. ConstructClusterTree tests level > l_max and recurses with l_max + 1;
  read as "split iff level < l_max", so all leaves sit at l_max (Sec. 3.2 says so).
* A point on a splitting plane goes to the lower half: the algorithm's halves
  are [alpha, mid] and (mid, beta].
* The 2^d children are enumerated by the little-endian child id
  c = sum_k b_k 2^(k-1), b_k = 1 for the upper half of axis k (axis 1 least
  significant, as the reshape convention of Sec. 2.1).
* Children whose box holds no point are not created (the paper is silent);
  this changes no matrix entry.
* Admissibility: max(diam) <= eta * dist is evaluated exactly, in rational
  arithmetic on the (dyadic, exactly representable) box bounds, with equality
  counting as admissible (the inequality is non-strict).  The distance formula's
  parenthesisation is read with both max-terms inside the sum over axes.
* Node ids are breadth-first: by level, then parent id, then child id.  Block
  lists are sorted by (level, sigma id, tau id).  Translation classes are keyed
  by (level, o) with o = k_tau - k_sigma the integer box offset, sorted by level
  then o lexicographically (axis 1 first).
"""

from fractions import Fraction

import numpy as np


class ClusterTree:
    """Nodes in breadth-first order.

    Attributes (lists indexed by node id):
      level, coords (tuple of ints, box index at its level), lo, hi (float box
      bounds per axis), idx (original point indices in order), parent (-1 for
      the root), children (list of node ids ordered by child id), cid (child id
      within the parent).
    Also: leaves (leaf ids in tree order), perm (tree position -> original
    index), begin/end (range of a node in tree order), l_max, d, box_lo, box_hi.
    """


def build_cluster_tree(X, lo, hi, l_max):
    """Alg. ConstructClusterTree from the root box [lo, hi]^d with maximum level l_max."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    raw = []  # (level, coords, lo, hi, idx, parent_raw, cid)

    def make(level, coords, blo, bhi, idx, parent, cid):
        raw.append(dict(level=level, coords=coords, lo=blo, hi=bhi, idx=idx,
                        parent=parent, cid=cid, children=[]))
        return len(raw) - 1

    root = make(0, tuple([0] * d), np.full(d, float(lo)), np.full(d, float(hi)),
                np.arange(n, dtype=np.int64), -1, 0)

    def recurse(node):
        nd = raw[node]
        if nd["level"] >= l_max:
            return
        mid = (nd["lo"] + nd["hi"]) / 2.0
        pts = X[nd["idx"]]
        upper = pts > mid[None, :]            # lower half is [alpha, mid]
        cids = np.zeros(len(nd["idx"]), dtype=np.int64)
        for k in range(d):
            cids += upper[:, k].astype(np.int64) << k
        for c in range(2 ** d):
            sel = nd["idx"][cids == c]        # boolean mask keeps the parent's order
            if sel.size == 0:
                continue
            clo = nd["lo"].copy()
            chi = nd["hi"].copy()
            coords = list(nd["coords"])
            for k in range(d):
                if (c >> k) & 1:
                    clo[k] = mid[k]
                    coords[k] = 2 * coords[k] + 1
                else:
                    chi[k] = mid[k]
                    coords[k] = 2 * coords[k]
            ch = make(nd["level"] + 1, tuple(coords), clo, chi, sel, node, c)
            nd["children"].append(ch)
        for ch in nd["children"]:
            recurse(ch)

    recurse(root)

    # breadth-first renumbering: level, then parent id, then child id
    order = [root]
    head = 0
    while head < len(order):
        order.extend(raw[order[head]]["children"])
        head += 1
    new_id = {old: i for i, old in enumerate(order)}

    t = ClusterTree()
    t.d = d
    t.l_max = l_max
    t.box_lo = float(lo)
    t.box_hi = float(hi)
    t.level = [raw[o]["level"] for o in order]
    t.coords = [raw[o]["coords"] for o in order]
    t.lo = [raw[o]["lo"] for o in order]
    t.hi = [raw[o]["hi"] for o in order]
    t.idx = [raw[o]["idx"] for o in order]
    t.parent = [new_id[raw[o]["parent"]] if raw[o]["parent"] >= 0 else -1 for o in order]
    t.children = [[new_id[c] for c in raw[o]["children"]] for o in order]
    t.cid = [raw[o]["cid"] for o in order]
    t.n_nodes = len(order)
    t.leaves = [i for i in range(t.n_nodes) if not t.children[i]]
    t.perm = np.concatenate([t.idx[i] for i in t.leaves]) if t.leaves else np.zeros(0, np.int64)
    # tree-order ranges: a node's points are contiguous in the leaf concatenation
    begin = [0] * t.n_nodes
    end = [0] * t.n_nodes
    pos = 0
    for i in t.leaves:
        begin[i] = pos
        pos += len(t.idx[i])
        end[i] = pos
    for i in reversed(range(t.n_nodes)):
        if t.children[i]:
            begin[i] = min(begin[c] for c in t.children[i])
            end[i] = max(end[c] for c in t.children[i])
    t.begin = begin
    t.end = end
    return t


def diam2(lo, hi):
    """Squared diameter of a hypercube (App. "Additional Definitions"), exact rational."""
    return sum((Fraction(float(b)) - Fraction(float(a))) ** 2 for a, b in zip(lo, hi))


def dist2(lo1, hi1, lo2, hi2):
    """Squared distance of two hypercubes (App. "Additional Definitions"), exact rational."""
    s = Fraction(0)
    for a, b, c, dd in zip(lo1, hi1, lo2, hi2):
        a, b, c, dd = (Fraction(float(v)) for v in (a, b, c, dd))
        s += max(Fraction(0), a - dd) ** 2 + max(Fraction(0), c - b) ** 2
    return s


def admissible(t, s, u, eta2):
    """Eq. "admissible": max(diam B_s, diam B_u) <= eta * dist(B_s, B_u), squared, exact.

    ``eta2`` is eta^2 as a Fraction (or int).
    """
    lhs = max(diam2(t.lo[s], t.hi[s]), diam2(t.lo[u], t.hi[u]))
    return lhs <= Fraction(eta2) * dist2(t.lo[s], t.hi[s], t.lo[u], t.hi[u])


def build_block_tree(t, eta2):
    """Alg. ConstructBlockClusterTree from root x root.

    Returns (near, far): lists of (sigma, tau) leaf blocks, sorted by
    (level, sigma, tau).  near = inadmissible leaves (set D), far = admissible
    leaves (set A).
    """
    near, far = [], []
    cache = {}

    def adm(s, u):
        key = (s, u)
        if key not in cache:
            cache[key] = admissible(t, s, u, eta2)
        return cache[key]

    stack = [(0, 0)]
    while stack:
        s, u = stack.pop()
        a = adm(s, u)
        if (not a) and t.children[s] and t.children[u]:
            for sc in t.children[s]:
                for uc in t.children[u]:
                    stack.append((sc, uc))
        elif a:
            far.append((s, u))
        else:
            near.append((s, u))
    key = lambda b: (t.level[b[0]], b[0], b[1])
    return sorted(near, key=key), sorted(far, key=key)


def translation_classes(t, far):
    """Sec. 5.2: far blocks of a stationary kernel share M_b when (level, offset) agree.

    Returns (classes, block_class): classes is the sorted list of keys
    (level, o) and block_class[i] is the class index of far[i].
    """
    keys = []
    for s, u in far:
        o = tuple(int(cu) - int(cs) for cs, cu in zip(t.coords[s], t.coords[u]))
        keys.append((t.level[s], o))
    classes = sorted(set(keys))
    pos = {k: i for i, k in enumerate(classes)}
    return classes, [pos[k] for k in keys]


def default_l_max(n, d, leaf_size):
    """Smallest l with n / 2^(d l) <= leaf_size (uniform depth; leaf size -> depth reading)."""
    l = 0
    while n > leaf_size * (2 ** (d * l)):
        l += 1
    return l
