"""Pins of the history operations in the CPU reference (Supp. "History Recovery",
alg:example; Supp. "Batched Updates"), on hand-written cases and on the round trip the
paper states: the recovered state equals the stored one exactly."""
import numpy as np

import oracle


def test_reorder_and_recover_by_hand():
    g = [np.array([10, 11, 12, 13, 14, 15]), np.array([[0, 1, 2, 3, 4, 5], [6, 7, 8, 9, 10, 11]])]
    ind = np.array([0, 1, 0, 0, 1, 0], bool)
    (a, b), ns = oracle.reorder_static_first(g, ind)
    assert ns == 4 and a.tolist() == [10, 12, 13, 15, 11, 14]
    assert b.tolist() == [[0, 2, 3, 5, 1, 4], [6, 8, 9, 11, 7, 10]]
    # optimisation changes the changed rows (and may add or remove some): G^t
    latest = [np.array([10, 12, 13, 15, 91, 92, 93]), np.array([[0, 2, 3, 5, 81, 82, 83], [6, 8, 9, 11, 71, 72, 73]])]
    o = [np.array([11, 14]), np.array([[1, 4], [7, 10]])]          # O^t: values before optimisation
    rec = oracle.recover_previous(latest, ind, o)
    assert rec[0].tolist() == g[0].tolist() and rec[1].tolist() == g[1].tolist()


def test_multi_step_recovery_round_trip():
    """Three steps, each changing a random subset and resizing the change set; recovering
    step by step from the latest state gives back every stored state bit for bit."""
    rng = np.random.default_rng(0)
    state = [rng.normal(size=(3, 50)).astype(np.float32), rng.normal(size=50).astype(np.float32)]
    states, history = [state], []
    for _ in range(3):
        n = state[1].shape[-1]
        ind = rng.random(n) < 0.3
        o = [a[..., ind] for a in state]
        (re, ns) = oracle.reorder_static_first(state, ind)
        m = int(rng.integers(1, 20))                                   # the change set after optimisation
        new = [np.concatenate([r[..., :ns], rng.normal(size=r.shape[:-1] + (m,)).astype(np.float32)], axis=-1)
               for r in re]
        history.append((ind, o))
        state = new
        states.append(state)
    cur = states[-1]
    for k in range(3, 0, -1):
        ind, o = history[k - 1]
        cur = oracle.recover_previous(cur, ind, o)
        for x, y in zip(cur, states[k - 1]):
            np.testing.assert_array_equal(x, y)


def test_merge_of_two_updates_by_hand():
    prev = [np.array([0, 1, 2, 3, 4, 5, 6])]
    i1 = np.array([0, 1, 1, 0, 0, 0, 0], bool)
    i2 = np.array([0, 0, 1, 0, 0, 1, 0], bool)
    out = oracle.merge_updates(prev, i1, i2, [np.array([21, 22, 23])], [np.array([31])])
    assert out[0].tolist() == [0, 3, 4, 6, 21, 22, 23, 31]
