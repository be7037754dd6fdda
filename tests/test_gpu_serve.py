"""Serving on the GPU: stored states rendered through gather lists equal renders of
naive snapshots, and every request gives the same image alone and in the mix (bit for
bit: the forward pass has no atomics and a fixed order)."""
import numpy as np
import pytest
import torch

import scenes
from paper_2506_21117_amd import api
from paper_2506_21117_amd.serve import Engine, GpuBackend, StateStore, poisson_requests

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def store_and_states():
    states, history = scenes.serving_history(seed=5, n_base=60_000, n_steps=4, delta_range=(2_000, 6_000))
    store = StateStore.from_history(states[-1], history)
    store.to_device(torch.device("cuda:0"))
    return store, states


def test_gathered_state_equals_snapshot(dev, store_and_states):
    store, states = store_and_states
    cam = scenes.sphere_camera(np.random.default_rng(2), 4.0, width=320, height=240, fx=330.0)
    be = GpuBackend(store, dev)
    for k in (0, 2, len(states) - 1):
        snap = api.GaussianTensors.from_scene(states[k], dev)
        proj = api.project_preprocess(snap, [cam])
        bins = api.bin_and_sort(proj, [cam], capacity=4_000_000, mode=api._ffi.BINS_COMPLETE)
        ref, _, _ = api.render_forward(proj, bins, [cam])
        from paper_2506_21117_amd.serve import Request
        got = be.render_alone(Request(0, k, cam))
        torch.cuda.synchronize()
        assert torch.equal(got, ref[0])


def test_alone_equals_mix(dev, store_and_states):
    store, states = store_and_states
    rng = np.random.default_rng(11)
    res = ((160, 120), (320, 240), (480, 360))
    reqs = poisson_requests(rng, 48, 2000.0, store.timesteps, res,
                            lambda r, w, h: scenes.sphere_camera(r, 4.0, width=w, height=h,
                                                                 fx=h / (2 * np.tan(np.radians(20)))))
    be = GpuBackend(store, dev, max_slots=4)
    eng = Engine(be, hbm_budget_bytes=2 << 30, max_slots=4, max_batch=4, keep_images=True)
    out, st = eng.run(reqs)
    torch.cuda.synchronize()
    s = st.summary()
    assert s["completed"] == len(reqs)
    assert s["groups"] < len(reqs)          # some requests shared a call
    assert s["peak_inflight"] >= 2          # work overlapped on the device
    by_id = {c.rid: c for c in out}
    for r in reqs:
        alone = be.render_alone(r)
        assert torch.equal(by_id[r.rid].image, alone), f"request {r.rid} differs alone vs in the mix"
    print(s)
