"""Cell-level definitions of SkyCell (Sections III and IV), written out on tiny grids.

TEST INFRASTRUCTURE ONLY: used by tests to pin the cell-pruning step; the product
path never imports it.

A layer with ``g`` columns per dimension has cells addressed by integer tuples
``c = (c[0], ..., c[d-1])``.  Tuples here are in dimension order 0..d-1; the
paper prints them from dimension d-1 down to 0 (Section III, grid structure).

Everything is plain Python over explicit cell tuples, so it is only meant for
grids of a few thousand cells.
"""
from itertools import product


def dominates_cell(a, b):
    """Definition 3: non-empty ``a`` dominates ``b`` iff a[k] < b[k] in every dimension.

    Emptiness is checked by the caller (the definition requires ``a`` to hold points).
    """
    return all(x < y for x, y in zip(a, b))


def partially_dominates_cell(a, b):
    """Definition 3: a[k] <= b[k] everywhere with equality in at least one dimension.

    A cell partially dominates itself.
    """
    return all(x <= y for x, y in zip(a, b)) and any(x == y for x, y in zip(a, b))


def dominated_cells(nonempty):
    """Cells (among ``nonempty``) dominated by another non-empty cell (Definition 3)."""
    ne = list(nonempty)
    return {b for b in ne if any(dominates_cell(a, b) for a in ne)}


def auxiliary_key_cells(g, d):
    """The d auxiliary key cells Lambda_j (Section IV-A).

    Auxiliary point lambda_j sits just below 1 in dimension j and just below 0
    elsewhere, so by Equation 1 its cell has column g-1 in dimension j and -1 in
    every other dimension.
    """
    return [tuple(g - 1 if k == j else -1 for k in range(d)) for j in range(d)]


def key_cells(nonempty, g, d, with_aux=True):
    """Definition 4: non-empty cells neither dominated nor partially dominated by any
    *other* cell.  With ``with_aux`` the auxiliary key cells take part as cells that
    can partially dominate (they are outside the grid, so they are returned separately).
    """
    ne = set(nonempty)
    others = list(ne) + (auxiliary_key_cells(g, d) if with_aux else [])
    keys = set()
    for c in ne:
        if any(o != c and (dominates_cell(o, c) or partially_dominates_cell(o, c)) for o in others):
            continue
        keys.add(c)
    return keys


def candidate_cells(nonempty, g, d):
    """Definition 5 / Equation 6 with the auxiliary key cells counted as key cells
    (the convention of the bijection proof of Theorem 1).

    C = K  union  Gamma(c) over key cells c, where Gamma(c) (Equation 5) holds the
    cells partially dominated by c and not dominated by any key cell.  Only cells
    of the grid are returned.
    """
    keys = key_cells(nonempty, g, d, with_aux=True)
    all_keys = list(keys) + auxiliary_key_cells(g, d)
    cand = set(keys)
    for c in product(range(g), repeat=d):
        if any(dominates_cell(k, c) for k in all_keys):
            continue
        if any(partially_dominates_cell(k, c) for k in all_keys):
            cand.add(c)
    return cand


def classify(nonempty, g, d):
    """Three cell types of Section III: 'dominated', 'candidate' or 'irrelevant'."""
    ne = set(nonempty)
    dom = dominated_cells(ne)
    cand = candidate_cells(ne, g, d)
    out = {}
    for c in product(range(g), repeat=d):
        if c in dom:
            out[c] = "dominated"
        elif c in cand:
            out[c] = "candidate"
        else:
            out[c] = "irrelevant"
    return out


def auxiliary_candidate_cells(g, d):
    """Lemma 2 / Equation 7: cells with column g-1 in at least one dimension."""
    return {c for c in product(range(g), repeat=d) if any(x == g - 1 for x in c)}


def omega(c, ck):
    """Equation 8: highest dimension where ``c`` and key cell ``ck`` share a column."""
    return max(j for j in range(len(c)) if c[j] == ck[j])


def big_omega(c, keys_with_aux):
    """Equation 9: minimum of omega over the key cells that partially dominate ``c``."""
    return min(omega(c, k) for k in keys_with_aux if partially_dominates_cell(k, c))


def psi(c, keys_with_aux, g):
    """Equation 10: map a candidate cell to an auxiliary candidate cell."""
    j = big_omega(c, keys_with_aux)
    return tuple(g - 1 if k == j else c[k] for k in range(len(c)))


def gamma_dim(ca, g):
    """Equation 12: smallest dimension where ``ca`` has column g-1."""
    return min(j for j in range(len(ca)) if ca[j] == g - 1)


def phi(ca, keys_with_aux, g):
    """Equation 13: smallest column, in dimension gamma(ca), of the key cells that are
    <= ca up to gamma(ca) and < ca above it."""
    gd = gamma_dim(ca, g)
    vals = [k[gd] for k in keys_with_aux
            if all(k[j] <= ca[j] for j in range(gd + 1))
            and all(k[j] < ca[j] for j in range(gd + 1, len(ca)))]
    return min(vals)


def theta(ca, keys_with_aux, g):
    """Equation 11: map an auxiliary candidate cell back to a candidate cell."""
    gd = gamma_dim(ca, g)
    ph = phi(ca, keys_with_aux, g)
    return tuple(ph if k == gd else ca[k] for k in range(len(ca)))


def candidate_count_closed_form(g, d):
    """Corollary 1 / Equation 14 with 2^i replaced by g: sum_j (g-1)^j g^(d-1-j)."""
    return sum((g - 1) ** j * g ** (d - 1 - j) for j in range(d))


def candidate_volume_fraction(g, d):
    """Corollary 2: fraction of the layer covered by candidate cells, 1 - (1 - 1/g)^d."""
    return 1.0 - (1.0 - 1.0 / g) ** d


# ---------------------------------------------------------------------------
# Parallel ShrinkKeyCells (Section V-B, Algorithm 3) and the layer loop of
# Algorithm 1, written out in the paper's order with numpy arrays standing in
# for the tree levels.  Cells are integer column tuples of one layer, held as
# rows of an [N, d] array; a pointer is a row number, -1 the padding leaf of a
# complete binary tree.
#
# These reproduce what the algorithm computes, including where it departs from
# the definitions: the tree keeps ONE pointer per node, and a cell can have
# several incomparable non-empty cells below it, so the pointer that reaches a
# leaf may be a partial dominator while a (strict) dominator exists elsewhere.
# Its "dominated" verdicts are always true (the pointer it holds dominates the
# cell), but some dominated cells come out as candidate or key cells; see
# tests/test_oracle.py for the three-cell counterexample in two dimensions.
# ---------------------------------------------------------------------------
import numpy as _np


def _rotated(cells, m):
    """Columns under rotation m: dimension k of the rotated cell is dimension
    (k + m) mod d of the cell (each rotation turns dimension k into k - 1 and
    dimension 0 into d - 1)."""
    d = cells.shape[1]
    return cells[:, [(k + m) % d for k in range(d)]]


def _k_dominates(cells, nonempty, a, b, k, m):
    """Vector form of 'cell a k-dominates cell b' under rotation m: a holds
    points, a <= b in every dimension, and a equals b in rotated dimensions
    k..d-1.  a, b: arrays of row numbers (>= 0)."""
    ra = _rotated(cells[a], m)
    rb = _rotated(cells[b], m)
    le = (ra <= rb).all(axis=1)
    eq = (ra[:, k:] == rb[:, k:]).all(axis=1)
    return nonempty[a] & le & eq


def _dom2(cells, nonempty, a, b, m):
    """dom_2(a, b): a if a 2-dominates b, else b; a padding pointer loses to any
    cell and a cell wins over a padding pointer."""
    out = b.copy()
    both = (a >= 0) & (b >= 0)
    aonly = (a >= 0) & (b < 0)
    out[aonly] = a[aonly]
    idx = _np.nonzero(both)[0]
    if idx.size:
        win = _k_dominates(cells, nonempty, a[idx], b[idx], 2, m)
        out[idx[win]] = a[idx[win]]
    return out


def shrink_key_cells_parallel(cells, nonempty):
    """Algorithm 3 on the cells `cells` ([N, d] columns of one layer, the split
    of the previous layer's candidate cells) with their occupancy `nonempty`.

    Returns (o, l): o[j] is the row of the j-th leaf in the final order and l[j]
    the row its l pointer names.  The caller classifies (Theorem 2): a key cell
    when l = o, a candidate when l partially dominates o.
    """
    cells = _np.asarray(cells, dtype=_np.int64)
    nonempty = _np.asarray(nonempty, dtype=bool)
    n, d = cells.shape
    if n == 0:
        return _np.zeros(0, _np.int64), _np.zeros(0, _np.int64)
    h = max(1, int(n - 1).bit_length())
    size = 1 << h
    o = _np.arange(n, dtype=_np.int64)
    l = o.copy()
    for m in range(max(1, d - 1)):
        # reorder the leaves by their columns under rotation m, dimension d-1
        # most significant (the leaves carry their pointers with them)
        r = _rotated(cells[o], m)
        order = _np.lexsort([r[:, k] for k in range(d)])
        o = o[order]
        l = l[order]
        u0 = o.copy() if m == 0 else l.copy()
        # bottom-up: u of a node is dom_2 of its children's u
        U = [_np.concatenate([u0, -_np.ones(size - n, _np.int64)])]
        for j in range(1, h + 1):
            prev = U[-1]
            U.append(_dom2(cells, nonempty, prev[0::2], prev[1::2], m))
        # top-down: l of a node from its parent's left neighbour and its own u
        Lrow = U[h].copy()
        for j in range(h - 1, -1, -1):
            cnt = U[j].size
            row = _np.empty(cnt, _np.int64)
            k = _np.arange(cnt)
            row[0] = U[j][0]
            odd = k[1::2]
            row[odd] = Lrow[(odd - 1) // 2]
            even = k[2::2]
            if even.size:
                row[even] = _dom2(cells, nonempty, Lrow[even // 2 - 1], U[j][even], m)
            Lrow = row
        l = Lrow[:n]
    return o, l


def classify_parallel(cells, nonempty):
    """Theorem 2 applied to the result of Algorithm 3: for every row of `cells`,
    'key' (l = o), 'candidate' (l partially dominates o) or 'dominated' (l
    dominates o); a cell whose l pointer is none of these is 'irrelevant'.
    Key cells must hold points."""
    cells = _np.asarray(cells, dtype=_np.int64)
    nonempty = _np.asarray(nonempty, dtype=bool)
    o, l = shrink_key_cells_parallel(cells, nonempty)
    out = _np.empty(cells.shape[0], dtype=object)
    for oi, li in zip(o.tolist(), l.tolist()):
        a, b = tuple(cells[li]), tuple(cells[oi])
        if li == oi:
            out[oi] = "key" if nonempty[oi] else "irrelevant"
        elif nonempty[li] and dominates_cell(a, b):
            out[oi] = "dominated"
        elif nonempty[li] and partially_dominates_cell(a, b):
            out[oi] = "candidate"
        else:
            out[oi] = "irrelevant"
    return out


def layers_parallel(coords_by_layer, rho, d):
    """The layer loop of Algorithm 1 with parallel ShrinkKeyCells: layer 0 is one
    cell (the whole space), a key and candidate cell; layer i+1 takes the 2^d
    children of every candidate cell of layer i (key cells included) as the
    leaves of Algorithm 3, and keeps its key and candidate cells.

    coords_by_layer(i) returns the set of non-empty cells (tuples) of layer i.
    Returns a list, per layer 0..rho, of dicts cell -> 'key' | 'candidate'.
    """
    result = [{(0,) * d: "key"}]
    cand = [(0,) * d]
    for i in range(rho):
        ne_set = coords_by_layer(i + 1)
        kids = []
        for c in cand:
            for s in product((0, 1), repeat=d):
                kids.append(tuple(2 * c[k] + s[k] for k in range(d)))
        if not kids:
            result.append({})
            cand = []
            continue
        arr = _np.array(kids, dtype=_np.int64)
        ne = _np.array([k in ne_set for k in kids], dtype=bool)
        cls = classify_parallel(arr, ne)
        layer = {kids[j]: cls[j] for j in range(len(kids)) if cls[j] in ("key", "candidate")}
        result.append(layer)
        cand = list(layer.keys())
    return result
