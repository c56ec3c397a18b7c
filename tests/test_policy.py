"""Relabel victim policy in the all-frame demand model (host only, no GPU).

Corollary 1 (Section IV-D) is the Belady rule for this setting: when the whole
fused stream is known, choosing as victim the frame that is needed again last
gives the fewest demand promotions.  Pinned by brute force over every eviction
choice on tiny streams; first-free and LRU can only do as well or worse.
"""
import functools
import itertools

import numpy as np
import pytest


@pytest.fixture(scope="module")
def P():
    import paper_2608_16940_amd as P
    P.lib()
    return P


def brute_force_min(n, frames, tuples):
    """Minimum promotions over all eviction choices (depth-first search with memo)."""
    tuples = [tuple(t) for t in tuples]

    @functools.lru_cache(maxsize=None)
    def best(i, frame_qubits):
        if i == len(tuples):
            return 0
        cur = tuples[i]
        missing = [q for q in cur if q not in frame_qubits]
        # every sequence of victim choices for the missing targets, in tuple order
        results = []

        def rec(fq, rest, cost):
            if not rest:
                results.append(cost + best(i + 1, fq))
                return
            eligible = [f for f in range(frames) if fq[f] not in cur]
            for f in eligible:
                nfq = list(fq)
                nfq[f] = rest[0]
                rec(tuple(nfq), rest[1:], cost + 1)

        rec(frame_qubits, missing, 0)
        return min(results)

    return best(0, tuple(range(frames)))


def random_stream(rng, n, frames, length):
    out = []
    for _ in range(length):
        k = int(rng.integers(1, frames + 1))
        out.append(tuple(int(q) for q in rng.choice(n, size=k, replace=False)))
    return out


@pytest.mark.parametrize("n,frames,length", [(4, 2, 6), (5, 3, 7), (6, 3, 8), (6, 4, 6), (5, 2, 8)])
def test_belady_is_optimal_brute_force(P, n, frames, length):
    rng = np.random.default_rng(100 * n + 10 * frames + length)
    for _ in range(12):
        s = random_stream(rng, n, frames, length)
        opt = brute_force_min(n, frames, s)
        bel = P.policy_simulate(n, frames, s, "belady")
        ff = P.policy_simulate(n, frames, s, "first_free")
        lru = P.policy_simulate(n, frames, s, "lru")
        assert bel == opt, (s, bel, opt)
        assert ff >= opt and lru >= opt


def test_policy_counts_simple_cases(P):
    # everything already in frames: no promotions
    assert P.policy_simulate(6, 3, [(0, 1), (2,), (1, 2, 0)], "belady") == 0
    # cyclic access over frames+1 qubits: after the three initial hits LRU misses
    # every access, farthest-next-use about one in three
    s = [(q % 4,) for q in range(12)]
    assert P.policy_simulate(6, 3, s, "lru") == 9
    assert P.policy_simulate(6, 3, s, "belady") == brute_force_min(6, 3, s) < 9


def test_policy_rejects_bad_input(P):
    with pytest.raises(P.SvError):
        P.policy_simulate(4, 2, [(0, 1, 2)], "belady")
    with pytest.raises(P.SvError):
        P.policy_simulate(4, 5, [(0,)], "belady")
