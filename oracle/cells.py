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
