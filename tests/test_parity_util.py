"""The GPU-vs-oracle parity check itself, exercised on the CPU with oracle results standing in
for a device's: identical results pass, a result that differs outside the logged
near-threshold decisions fails, and a result that follows one near decision taken the other
way passes through the oracle's replay of that decision."""
import numpy as np

import oracle as O
from parity_util import check_search


def test_identical_results_pass(small_index, small_workload):
    ora = O.search(small_index, small_workload["queries"][:20], 10, 8, 0.1)
    r = check_search(ora["ids"], ora["dists"].astype(np.float32), ora, small_index)
    assert not r["bad"] and r["same"] == 20


def test_unlogged_difference_fails(small_index, small_workload):
    ix = small_index
    ora = O.search(ix, small_workload["queries"][:5], 10, 8, 0.1)
    ids, d = ora["ids"].copy(), ora["dists"].copy()
    # replace the last result of query 0 by a far candidate: its distance is exact for that
    # vector, but the id is nowhere near a threshold of the oracle's search
    far = int(np.argmax(O.sq_dist_direct(ix["Y"], ora["qrot"][0])))
    assert far not in ora["near"][0]
    ids[0, -1] = far
    d[0, -1] = O.sq_dist_direct(ix["Y"][[far]], ora["qrot"][0])[0]
    d[0] = np.sort(d[0])
    ids[0] = ids[0][np.argsort(np.r_[ora["dists"][0][:-1], d[0, -1]], kind="stable")]
    r = check_search(ids, d.astype(np.float32), ora, ix)
    assert [b[0] for b in r["bad"]] == [0]


def test_wrong_distance_fails(small_index, small_workload):
    ora = O.search(small_index, small_workload["queries"][:5], 10, 8, 0.1)
    d = ora["dists"].copy()
    d[2, 3] *= 1 + 3e-4
    d[2] = np.sort(d[2])
    r = check_search(ora["ids"], d, ora, small_index)
    assert [b[0] for b in r["bad"]] == [2]


def test_one_flipped_near_decision_passes_by_replay(small_index, small_workload):
    """A device result equal to the search with one logged near decision taken the other way
    (here with a wide near tolerance so that such decisions exist) is accepted, through the
    replay, even where the flip changed tau for later blocks."""
    ix = small_index
    Q = small_workload["queries"][:30]
    ora = O.search(ix, Q, 10, 8, 0.1, near_tol=0.05)
    found = 0
    for qi in range(Q.shape[0]):
        for x in ora["stage_near"][qi][:6]:
            alt = O.search(ix, Q[qi:qi + 1], 10, 8, 0.1, near_tol=0.05, flip={0: [x]})
            if np.array_equal(alt["ids"][0], ora["ids"][qi]):
                continue
            one = dict(ora, ids=ora["ids"][qi:qi + 1], dists=ora["dists"][qi:qi + 1],
                       near=[ora["near"][qi]], stage_near=[ora["stage_near"][qi]],
                       probe_near=[ora["probe_near"][qi]], qrot=ora["qrot"][qi:qi + 1],
                       queries=Q[qi:qi + 1])
            r = check_search(alt["ids"], alt["dists"], one, ix)
            assert not r["bad"], r["bad"]
            assert r["excused"] == 1
            found += 1
            break
    assert found >= 3
