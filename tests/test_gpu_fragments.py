"""Detached fragments on the GPU against the oracle: labels (smallest node id
of each connected component of the alive springs) and the fragment and
detached counts must agree exactly, for random breakage patterns on the
workload graph and through the Lagrangian update with tracking on."""
import numpy as np
import pytest

import oracle as O
from oracle import step as S
from paper_1302_3663_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda:0").contiguous()


def gpu_fragments(ctx):
    import ctypes
    label = torch.zeros(max(ctx.eta, 1), dtype=torch.int32, device="cuda:0")
    nf, nd = ctypes.c_int(), ctypes.c_int()
    ctx._c(ctx.lib.ibb_fragments(ctx.ctx, ctypes.c_void_p(label.data_ptr()), ctypes.byref(nf), ctypes.byref(nd)),
           "ibb_fragments")
    torch.cuda.synchronize()
    return label.cpu().numpy()[:ctx.eta], nf.value, nd.value


_MAKERS = {
    "tube3d_64x64x128": lambda: synth.WORKLOADS["tube3d_64x64x128"](),
    "channel2d_64x32": lambda: synth.channel_2d(seed=1),
    "3d_tube": lambda: synth.tiny_3d(),
    "2d_inout_walls": lambda: synth.tiny_2d(inout=True),
}
_CACHE = {}


def case_of(name):
    if name not in _CACHE:
        _CACHE[name] = _MAKERS[name]()
    c = _CACHE[name]
    return dict(c, params=dict(c["params"]))


CASES = _MAKERS


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("frac", [1.0, 0.5, 0.1, 0.0])
def test_random_breakage(name, frac):
    from paper_1302_3663_amd import ibmg
    case = case_of(name)
    print("case", name, "alive fraction", frac, flush=True)
    ctx = ibmg.from_case(case)
    ij = case["ij"]
    alive = (np.random.default_rng(7).random(ij.shape[1]) < frac).astype(np.uint8)
    ctx.set_springs(dev(ij, torch.int32), dev(case["rest"], torch.float64), dev(case["K"], torch.float64),
                    dev(alive, torch.uint8))
    lab, nf, nd = gpu_fragments(ctx)
    olab, onf, ond = O.fragments(ij, alive, O.anchored_nodes(case["params"], case["X"]))
    assert np.array_equal(lab, olab)
    assert (nf, nd) == (onf, ond)
    ctx.close()


def test_no_springs():
    from paper_1302_3663_amd import ibmg
    case = synth.tiny_3d()
    case["ij"] = np.zeros((2, 0), np.int32)
    case["rest"] = np.zeros(0)
    case["K"] = np.zeros(0)
    ctx = ibmg.from_case(case)
    lab, nf, nd = gpu_fragments(ctx)
    n = case["X"].shape[1]
    anchored = O.anchored_nodes(case["params"], case["X"])
    assert np.array_equal(lab, np.arange(n)) and nf == n and nd == n - int(anchored.sum())
    ctx.close()


@pytest.mark.parametrize("name", ["3d_tube", "channel2d_64x32"])
def test_tracked_lagrangian_update(name):
    """Springs break at any stretch (break ratio just above 1); after each
    update the counts and labels match the oracle's step."""
    from paper_1302_3663_amd import ibmg
    case = case_of(name)
    case["params"] = dict(case["params"], break_ratio=1.0 + 1e-6, track_fragments=1)
    ctx = ibmg.from_case(case)
    st = S.State(case["params"], case["u0"], case["p0"], case["X"], case["ij"], case["rest"], case["K"])
    S.setup(st)
    for k in range(3):
        ctx.projection_step()
        S.projection_step(st)
        lg = ctx.lagrangian_update()
        lo = S.lagrangian_update(st)
        print("step", k, lg, {q: lo[q] for q in ("n_broken", "n_alive", "n_fragments", "n_detached")}, flush=True)
        assert lg["n_broken"] == lo["n_broken"] and lg["n_alive"] == lo["n_alive"]
        assert lg["n_fragments"] == lo["n_fragments"] and lg["n_detached"] == lo["n_detached"]
        lab, nf, nd = gpu_fragments(ctx)
        assert np.array_equal(lab, lo["label"]) and nf == lo["n_fragments"]
    assert lo["n_broken"] > 0 or st.alive.sum() < len(st.alive)
    ctx.close()


def test_untracked_stats_are_marked():
    from paper_1302_3663_amd import ibmg
    ctx = ibmg.from_case(synth.tiny_3d())
    ctx.projection_step()
    lg = ctx.lagrangian_update()
    assert lg["n_fragments"] == -1 and lg["n_detached"] == -1
    ctx.close()
