"""Textbook generalized arc consistency by enumeration, for tiny inputs only.

A value a of x_i is supported iff some point of the Cartesian product of the
current domains that has a in position i belongs to the relation (the GAC
definition at the start of Sec. 2 of the paper).  This module does not use
bitsets, supports or currTable: it enumerates the product and tests
membership in the tuple set, so it is independent of the oracle.
"""
from __future__ import annotations

import itertools


def gac(tuples, lo, dom_sets):
    """dom_sets: per variable a set of value offsets (v - lo_i).

    Returns (failed, out_sets, valid_indices) where valid_indices are the
    positions j of the tuples list whose every value lies in the domains.
    """
    n = len(dom_sets)
    rel = {}
    for j, tp in enumerate(tuples):
        key = tuple(int(tp[i]) - int(lo[i]) for i in range(n))
        rel.setdefault(key, []).append(j)
    keep = [set() for _ in range(n)]
    valid = []
    for point in itertools.product(*[sorted(s) for s in dom_sets]):
        js = rel.get(tuple(point))
        if js:
            valid.extend(js)
            for i, a in enumerate(point):
                keep[i].add(a)
    valid.sort()
    if not valid:
        return True, None, []
    return False, keep, valid


def closure(tables, scopes, pool_sets):
    """Largest sub-domains of ``pool_sets`` that are GAC for every table, by
    repeating per-table enumeration until nothing changes.  Returns
    (failed, pool_sets_out)."""
    pool = [set(s) for s in pool_sets]
    changed = True
    while changed:
        changed = False
        for (tuples, lo), scope in zip(tables, scopes):
            failed, out, _ = gac(tuples, lo, [pool[v] for v in scope])
            if failed:
                return True, None
            for k, v in enumerate(scope):
                if out[k] != pool[v]:
                    pool[v] = out[k]
                    changed = True
    return False, pool


STAR = -(1 << 31)  # a cell of a short table: any value of its column


def gac_short(tuples, lo, dom_sets):
    """Short table (cells may be STAR): a tuple is valid iff every cell is
    STAR or names a value of the domain; GAC by enumerating the product and
    testing each point against every tuple.  Returns (failed, out_sets,
    valid_indices)."""
    n = len(dom_sets)
    rows = [[None if int(tp[i]) == STAR else int(tp[i]) - int(lo[i]) for i in range(n)] for tp in tuples]
    keep = [set() for _ in range(n)]
    any_point = False
    for point in itertools.product(*[sorted(s) for s in dom_sets]):
        if any(all(c is None or c == p for c, p in zip(r, point)) for r in rows):
            any_point = True
            for i, a in enumerate(point):
                keep[i].add(a)
    valid = [j for j, r in enumerate(rows)
             if all((c is None and dom_sets[i]) or (c is not None and c in dom_sets[i]) for i, c in enumerate(r))]
    if not any_point:
        return True, None, []
    return False, keep, valid


def gac_negative(tuples, lo, dom_sets):
    """Negative table: the tuples are forbidden; a point of the product is
    allowed iff it is not listed.  Returns (failed, out_sets,
    listed_indices_in_the_product_of_out_sets)."""
    n = len(dom_sets)
    listed = {tuple(int(tp[i]) - int(lo[i]) for i in range(n)) for tp in tuples}
    keep = [set() for _ in range(n)]
    any_point = False
    for point in itertools.product(*[sorted(s) for s in dom_sets]):
        if point not in listed:
            any_point = True
            for i, a in enumerate(point):
                keep[i].add(a)
    if not any_point:
        return True, None, []
    valid = [j for j, tp in enumerate(tuples)
             if all(int(tp[i]) - int(lo[i]) in keep[i] for i in range(n))]
    return False, keep, valid
