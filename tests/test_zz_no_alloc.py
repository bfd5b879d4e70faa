"""GPU: the allocation-free energy histogram (pic_spectrum_counts_noalloc)
through the C ABI against the allocating entry point, on two calls in a row,
the second with fewer edges and a narrower x range (the staging keeps the
previous call's contents, so what must start at zero is cleared per call).
The counts are integers: bit-exact equality."""

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2502_13695_amd import pic
    pic.lib()
    return pic


@pytest.mark.parametrize("which", ["config_2d", "config_3d"])
def test_noalloc_histogram_equals_allocating_one(P, which):
    cfg = getattr(W, which)(**({"nx": 256, "ny": 64} if which == "config_2d" else {"nx": 96, "ny": 16, "nz": 16,
                                                                                   "front": 24}))
    ndim = cfg["ndim"]
    st = W.random_state(cfg, 40000, seed=55, e_scale=1e8)
    rng = np.random.default_rng(56)
    d = st["u"] / np.linalg.norm(st["u"], axis=1, keepdims=True)
    st["u"] = (d * (10.0 ** rng.uniform(-4.0, 0.5, len(d)))[:, None]).astype(np.float32)
    rec = np.zeros(len(st["kind"]), dtype=P.PARTICLE_DTYPE)
    rec["cell"][:, :ndim] = st["cell"][:, :ndim]
    rec["off"] = st["off"]
    rec["u"] = st["u"]
    rec["kind"] = st["kind"]
    ctx = P.Context(cfg)
    ctx.set_state(0, st["E"], st["b"], rec)
    calls = [(np.geomspace(1e-4, 3e6, 3001), 0, 0),            # counts through HBM atomics
             (np.geomspace(1e-3, 1e5, 120), 30, 70)]           # fewer edges, LDS counts, x range
    for edges, lo, hi in calls:
        want = ctx.spectrum(edges, lo, hi)
        got = ctx.spectrum_noalloc(edges, lo, hi)
        assert got.shape == want.shape
        assert np.array_equal(got, want)
        assert int(got.sum()) > 0
    # after a few steps (births and moves), once more
    ctx.step(3)
    edges = np.geomspace(1e-2, 1e4, 64)
    assert np.array_equal(ctx.spectrum_noalloc(edges), ctx.spectrum(edges))
    # beyond the staging's maximum: refused
    with pytest.raises(P.PicError) as e:
        ctx.spectrum_noalloc(np.geomspace(1e-3, 1e5, 4098))
    assert e.value.code == -1
    ctx.close()
