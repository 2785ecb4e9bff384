"""Host-only checks of the factorisation's task order (the ticket order of the
persistent factor launch, read back through the rr_factor_schedule hook).

The unpivoted band LU of a block-banded matrix with B tiles each side of the
diagonal (the no-fill factorisation the method's direct solves rest on,
Sec. 3.1) updates tile (r, t) as A_rt -= sum_s L_rs U_st over
s in [max(0, max(r, t) - B), min(r, t) - 1], then finalises it against the
LU of diagonal tile m = min(r, t).  The launch splits each off-diagonal tile
into an early task E (all updates but the last, written as a partial tile)
and a final task F (the last update, the triangular solve, and for distances
up to three a chain tile with the full inverse of tile m); a diagonal tile's
early updates are split into E' (s <= m - 3) and G (s = m - 2, on top of
E'), and the tile is factored by a worker of its own (s = m - 1, then the
LU); two more ticket tasks form its chain tiles.  The waits each task makes
are restated here from the kernel:

  E(r, t)        waits on the final L_rs, U_st of its early updates;
  E'(m, m)       waits on the final L_ms, U_sm, s <= m - 3;
  G(m, m)        waits on E'(m, m) and the final L_m,m-2, U_m-2,m;
  F(r, t)        waits on E(r, t), the final L_rs, U_st of s = m - 1, the
                 block-inverse LU of diagonal tile m, and (distance <= 3) the
                 full inverse of tile m;
  diagonal m     (worker, in order m = 0, 1, ...) waits on G(m, m) and the
                 final L_m,m-1, U_m-1,m;
  chain task m   waits on the full inverse of tile m and reads the final
                 tiles (m, m - d), (m - d, m) for d <= 3 without a wait of
                 its own, so those must be ordered before it through the
                 flags it does wait on.

Checked: every task appears exactly once; one ticket worker beside the
diagonal worker finishes the whole order (so no residency can deadlock it:
the smallest unfinished ticket never waits on a larger one); and every tile a
task reads is final by a chain of flag waits."""
import ctypes

import numpy as np
import pytest

from paper_1902_01458_amd import _lib

CHAIN_D = 3  # chain tiles are formed for distances 1 .. 3
F, E, CHAIN_L, CHAIN_U, EDIAG, GDIAG = 0, 1, 2, 3, 4, 5  # task kinds


def schedule(B, NB):
    L = _lib.lib()
    n = L.rr_factor_schedule(B, NB, None, 0)
    assert n >= 0
    out = (ctypes.c_int32 * max(1, 3 * n))()
    assert L.rr_factor_schedule(B, NB, out, n) == n
    return [tuple(out[3 * i:3 * i + 3]) for i in range(n)]


def band_tiles(B, NB):
    return [(r, t) for r in range(NB) for t in range(NB) if r != t and abs(r - t) <= B]


def update_range(r, t, B):
    return max(0, max(r, t) - B), min(r, t) - 1


def early_range(r, t, B):
    lo, hi = update_range(r, t, B)
    return lo, hi - 1


def has_early(r, t, B):
    lo, hi = early_range(r, t, B)
    return lo <= hi


def ediag_range(m, B):
    return max(0, m - B), m - 3


def has_ediag(m, B):
    lo, hi = ediag_range(m, B)
    return lo <= hi


CASES = [(B, NB) for B in (1, 2, 3, 4, 5, 8, 11) for NB in sorted({1, 2, 3, B, B + 1, 2 * B + 3, 24})]


def test_rejects_bad_sizes():
    L = _lib.lib()
    assert L.rr_factor_schedule(0, 4, None, 0) == -1
    assert L.rr_factor_schedule(3, 0, None, 0) == -1


@pytest.mark.parametrize("B,NB", CASES)
def test_every_task_once(B, NB):
    tasks = schedule(B, NB)
    assert len(set(tasks)) == len(tasks)
    want = {(F, r, t) for r, t in band_tiles(B, NB)}
    want |= {(E, r, t) for r, t in band_tiles(B, NB) if has_early(r, t, B)}
    want |= {(EDIAG, m, m) for m in range(NB) if has_ediag(m, B)}
    want |= {(GDIAG, m, m) for m in range(NB) if has_early(m, m, B)}
    want |= {(k, m, m) for m in range(1, NB) for k in (CHAIN_L, CHAIN_U)}
    assert set(tasks) == want


@pytest.mark.parametrize("B,NB", CASES)
def test_one_worker_finishes_and_reads_are_ordered(B, NB):
    tasks = schedule(B, NB)
    # knowledge of a publish: the set of final (or partial) tile versions that
    # happen before it, as a bitset over (kind, r, t) keys
    keys = {}

    def bit(key):
        if key not in keys:
            keys[key] = len(keys)
        return 1 << keys[key]

    final = {}      # (r, t) -> knowledge at its final publish (diagonal: LU published)
    partial = {}    # (r, t) -> knowledge at E's publish (diagonal: E-prime's)
    partial2 = {}   # (m, m) -> knowledge at G's publish
    dinv = {}       # m -> knowledge at the full-inverse publish

    def need_final(r, t):
        return final.get((r, t))

    def run_diagonal(m):
        """The diagonal worker's step m, if its inputs are published."""
        k = dinv[m - 1] if m >= 1 else 0
        if has_early(m, m, B):
            if (m, m) not in partial2:
                return False
            k |= partial2[(m, m)]
        if m >= 1:
            for key in ((m, m - 1), (m - 1, m)):
                if key not in final:
                    return False
                k |= final[key]
        final[(m, m)] = k | bit(("F", m, m))
        dinv[m] = final[(m, m)] | bit(("D", m, m))
        return True

    next_diag = 0

    def advance_diagonal():
        nonlocal next_diag
        while next_diag < NB and run_diagonal(next_diag):
            next_diag += 1

    for i, (kind, r, t) in enumerate(tasks):
        advance_diagonal()
        m = min(r, t)
        k = 0
        waits = []
        if kind in (E, EDIAG):
            lo, hi = early_range(r, t, B) if kind == E else ediag_range(m, B)
            waits = [("F", r, s) for s in range(lo, hi + 1)] + [("F", s, t) for s in range(lo, hi + 1)]
        elif kind == GDIAG:
            if has_ediag(m, B):
                waits.append(("E", m, m))
            waits += [("F", m, m - 2), ("F", m - 2, m)]
        elif kind == F:
            lo, hi = update_range(r, t, B)
            if has_early(r, t, B):
                waits.append(("E", r, t))
            if hi >= lo:
                waits += [("F", r, hi), ("F", hi, t)]
            waits.append(("F", m, m))
            if abs(r - t) <= CHAIN_D:
                waits.append(("D", m, m))
        else:
            waits.append(("D", m, m))
        for w, a, b in waits:
            if w == "E":
                got = partial.get((a, b))
            elif w == "G":
                got = partial2.get((a, b))
            elif w == "D":
                got = dinv.get(a)
            else:
                got = need_final(a, b)
            assert got is not None, f"ticket {i} {(kind, r, t)} waits on unpublished {(w, a, b)}"
            k |= got | bit((w, a, b))
        if kind in (E, EDIAG):
            partial[(r, t)] = k | bit(("E", r, t))
        elif kind == GDIAG:
            partial2[(r, t)] = k | bit(("G", r, t))
        elif kind == F:
            final[(r, t)] = k | bit(("F", r, t))
        else:
            # the chain task's reads without waits of their own
            for d in range(1, min(CHAIN_D, B, m) + 1):
                tile = (m, m - d) if kind == CHAIN_L else (m - d, m)
                assert k & bit(("F",) + tile), f"chain task {(kind, m)} reads {tile} unordered"
    advance_diagonal()
    assert next_diag == NB
    assert set(final) == {(r, t) for r, t in band_tiles(B, NB)} | {(m, m) for m in range(NB)}
