"""The parity tests' resolution of in-band decisions (gpu_common.
checked_reference / check_against), exercised on the CPU with results built
from the oracle itself: the default outcomes pass, the other outcome of every
in-band decision passes too and is recognised as such, and a colour that
matches neither outcome is rejected."""
import numpy as np
import pytest

from paper_2505_05587_amd import scenes
from tests.gpu_common import check_against, checked_reference, packed_index, s9_to_s6, scene_small


def _as_gpu(ref):
    return dict(image=ref["image"].copy(), T_final=ref["T_final"].copy(), n_used=ref["n_used"].copy(),
                grads=ref["grads"].copy(), S6=s9_to_s6(ref["S"]).copy())


@pytest.mark.parametrize("mode", ["3dgs", "smooth"])
def test_checked_reference_accepts_either_outcome(oracle, mode):
    P, deg, cams, target = scene_small("sh3_pinhole")
    opts = scenes.opts(mode)
    ref = oracle.forward_backward(P, deg, cams, opts, target)
    one = np.nonzero(ref["pix_ndec"] == 1)[0]
    assert len(one) >= 3
    # the default outcome everywhere
    g = _as_gpu(ref)
    st = check_against(g, checked_reference(oracle, P, deg, cams, opts, g, target=target), cams, "default")
    assert st["gpu_flipped"] == 0 and st["flagged"] >= len(one)
    # the other outcome of every single in-band decision
    e = packed_index(cams, one)
    nv = len(one)
    var = oracle.pixel_variants(P, deg, cams, opts, target, np.concatenate([one, one]),
                                np.concatenate([-np.ones(nv, np.int32), np.zeros(nv, np.int32)]),
                                np.full((2 * nv, 3), 2))
    g = _as_gpu(ref)
    for k, p in enumerate(one):
        g["image"][e[k]] = var["rgb"][nv + k]
        g["T_final"][p] = var["T_final"][nv + k]
        g["n_used"][p] = var["n_used"][nv + k]
        for sign, (gid, gr, Sv) in ((-1.0, var["terms"][k]), (1.0, var["terms"][nv + k])):
            g["grads"][:, gid] += sign * gr.T
            g["S6"][:, gid] += sign * s9_to_s6(Sv.T)
    vref = checked_reference(oracle, P, deg, cams, opts, g, target=target)
    st = check_against(g, vref, cams, "flipped")
    distinct = np.abs(var["rgb"][nv:] - var["rgb"][:nv]).max(axis=1) > 2e-5
    assert st["gpu_flipped"] >= distinct.sum()
    # a colour that fits neither outcome
    g["image"][e[0]] += 1e-3
    with pytest.raises(AssertionError, match="matches no outcome"):
        checked_reference(oracle, P, deg, cams, opts, g, target=target)
