"""Model check of the resident stepper's rim exchange (CPU).

The resident kernel keeps each tile's state on chip for a whole call and
trades rims through two buffers chosen by generation parity, each word
carrying its generation as a tag; the state is read from the caller's
buffers at the start of a call and written back in place at the end.  This
test runs that protocol as a model: tiles on a ring (each tile's halo comes
from both neighbours) are coroutines whose every memory action (initial
read, rim store, rim load, final write) is one scheduling point, and a random
scheduler interleaves them.  Under every schedule tried it checks that

* a load never returns the wanted tag with a value of another generation
  (two parity buffers suffice: a word of generation g is only overwritten by
  g + 2 after every reader took g),
* no tile writes its result in place before each neighbour finished its
  initial read of it (a call runs at least two generations),
* every tile finishes (no wait goes unanswered when all tiles run).

A variant with one buffer instead of two, and one that allows a call of a
single generation, must fail the first and second checks: the model would
catch those mistakes.
"""
from __future__ import annotations

import random

import pytest


def run(ntiles, n, seed, buffers=2, min_gens=2):
    rng = random.Random(seed)
    # rim[parity][tile] = (tag, value): value is the (tile, generation) pair
    # that wrote it, standing in for the data
    rim = [[(0, None)] * ntiles for _ in range(buffers)]
    read_initial = [set() for _ in range(ntiles)]   # tiles that read my initial cells
    errors = []

    def tile(t):
        left, right = (t - 1) % ntiles, (t + 1) % ntiles
        # initial read of the caller's buffers: own cells and the neighbours' edge cells
        for nb in (left, right):
            read_initial[nb].add(t)
            yield
        gens = max(n, min_gens) if min_gens else n
        for g in range(1, gens + 1):
            # compute generation g from g - 1 (local), then publish unless last
            if g == gens:
                break
            par = g % buffers
            rim[par][t] = (g, (t, g))
            yield
            for nb in (left, right):
                while True:
                    tag, val = rim[par][nb]
                    yield
                    if tag == g:
                        if val != (nb, g):
                            errors.append(f"tile {t} read {val} for ({nb}, {g})")
                        break
                    if tag > g:
                        errors.append(f"tile {t} missed generation {g} of tile {nb} (found {tag})")
                        break
        # in-place final write: every neighbour must have read its initial halo
        for nb in (left, right):
            if nb not in read_initial[t]:
                errors.append(f"tile {t} wrote its result before tile {nb} read it")
        yield

    live = {t: tile(t) for t in range(ntiles)}
    steps = 0
    while live:
        t = rng.choice(list(live))
        try:
            next(live[t])
        except StopIteration:
            del live[t]
        steps += 1
        if steps > 200000:
            errors.append("no progress")
            break
    return errors


@pytest.mark.parametrize("ntiles", [2, 3, 5])
@pytest.mark.parametrize("n", [2, 3, 7])
def test_two_parity_buffers_and_in_place_write_are_safe(ntiles, n):
    for seed in range(60):
        assert run(ntiles, n, seed) == [], (ntiles, n, seed)


def test_model_catches_a_single_buffer():
    assert any(run(3, 9, seed, buffers=1) for seed in range(200))


def test_model_catches_a_one_generation_call_written_in_place():
    assert any(run(3, 1, seed, min_gens=0) for seed in range(200))
