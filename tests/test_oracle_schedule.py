"""Pins for the oracle's round-robin table (Section 3.2, Algorithm 1).

* Table 1 (Section 2.2) lists the K_6 colouring colour by colour; the
  oracle's table must reproduce it in order.
* Section 3.2's steps (ii) and (iv): each step's target set pairs the q-th
  index with the (p_even - q + 1)-th, and between steps the index vector turns
  by one place with its first entry fixed.  Rebuilding the index vector from
  each step of the table and checking that turn pins the slot order.
* Theorem 1 (Baranyai special case) and Section 3.2: p - 1 colours for even p,
  p for odd p; p/2 (even) or (p - 1)/2 (odd) real pairs per colour.
* An edge colouring: every edge of K_p appears exactly once per sweep, and
  no two pairs of one colour share a vertex (a matching).
"""
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "k6_table1.txt")


def _read_k6():
    cols = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        cols.append({frozenset((int(t[0]) - 1, int(t[1]) - 1)) for t in line.split()})
    return cols


def test_k6_matches_table1_in_order():
    want = _read_k6()
    tab = oracle.round_robin(6)
    got = [{frozenset(map(int, pr)) for pr in tab[k]} for k in range(tab.shape[0])]
    assert got == want


def _real_pairs(tab, p):
    out = []
    for k in range(tab.shape[0]):
        out.append([(int(a), int(b)) for a, b in tab[k] if a != p and b != p])
    return out


@pytest.mark.parametrize("p", list(range(1, 66)) + [100, 101, 257, 1000, 1001])
def test_round_robin_is_minimal_edge_colouring(p):
    tab = oracle.round_robin(p)
    pe = p + (p & 1)
    assert tab.shape == (pe - 1, pe // 2, 2)
    colours = _real_pairs(tab, p)
    # Colour count: p - 1 (even p) or p (odd p).
    assert len(colours) == (p - 1 if p % 2 == 0 else p)
    seen = np.zeros((p, p), dtype=np.int64)
    for pairs in colours:
        # Pairs per colour: p/2 or (p-1)/2.
        assert len(pairs) == p // 2
        verts = [v for pr in pairs for v in pr]
        assert len(verts) == len(set(verts))          # a matching
        for a, b in pairs:
            assert a != b and 0 <= a < p and 0 <= b < p
            seen[min(a, b), max(a, b)] += 1
    iu = np.triu_indices(p, 1)
    assert np.all(seen[iu] == 1)                       # every edge exactly once
    assert seen[np.tril_indices(p)].sum() == 0


@pytest.mark.parametrize("p", [5, 7, 9, 101])
def test_odd_p_dummy_pairs_with_every_vertex_once(p):
    # For odd p the dummy index p+1 (value p here) idles one real vertex per
    # colour (step iii); over a sweep each real vertex idles exactly once.
    tab = oracle.round_robin(p)
    idle = []
    for k in range(tab.shape[0]):
        for a, b in tab[k]:
            if a == p or b == p:
                idle.append(int(b) if a == p else int(a))
    assert sorted(idle) == list(range(p))


def test_first_table_is_identity_pairing():
    # Section 3.2 step (ii): the first target set is {1, pe}, {2, pe-1}, ...
    for p in (6, 8, 11):
        pe = p + (p & 1)
        tab = oracle.round_robin(p)
        want = [(q, pe - 1 - q) for q in range(pe // 2)]
        assert [tuple(map(int, x)) for x in tab[0]] == want


def _index_vector(tab_k, pe):
    # Step (ii): slot q (0-based) holds positions q and pe - 1 - q.
    v = np.empty(pe, dtype=np.int64)
    for q, (a, b) in enumerate(tab_k):
        v[q], v[pe - 1 - q] = a, b
    return v


@pytest.mark.parametrize("p", [2, 3, 4, 6, 7, 10, 33, 64, 101, 256])
def test_index_vector_turns_one_place_per_step(p):
    # Step (iv): after each step the last index moves to position 2 and
    # positions 2..pe-1 move one place right; position 1 never moves.  The
    # first vector is the identity (1..pe).
    pe = p + (p & 1)
    tab = oracle.round_robin(p)
    prev = _index_vector(tab[0], pe)
    assert np.array_equal(prev, np.arange(pe))
    for k in range(1, tab.shape[0]):
        cur = _index_vector(tab[k], pe)
        assert cur[0] == 0
        assert np.array_equal(cur[1:], np.roll(prev[1:], 1))
        prev = cur
