"""The allocation-free decode adjoint (gs_decode_backward_noalloc) against gs_decode_backward.

The two share their kernels; the no-alloc call takes the weight-gradient
partials from the library's per-GPU device array instead of a caller scratch
buffer.  Both sum the partials in the same fixed order, so every gradient
must be bit-identical.  Two calls in a row, the second on a smaller anchor
set (and another head), check that the array's leftover contents from the
first call do not leak into the second.
"""
import ctypes
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from gen import scenes as S  # noqa: E402

import paper_2503_11731_amd as gs  # noqa: E402
from paper_2503_11731_amd import _lib as L  # noqa: E402

DEV = torch.device("cuda:0")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case(kind, n_anchors, n_assets, seed):
    sc = S.corridor_anchors(seed=seed, n_anchors=n_anchors, sensor_kind=kind, z_lo=-20, z_hi=40,
                            n_assets=n_assets, asset_anchors=150)
    sensor = S.pinhole(320, 200, 160.0, pose=S.camera_yaw_pose(10.0)) if kind == "pinhole" else \
        S.lidar_spinning(n_beams=32, n_az=360)
    dec = gs.Decoder.from_gen(sc, DEV)
    sp = gs.poses_tensor(sensor["pose"], DEV)[0]
    gp = gs.poses_tensor(sc.group_poses, DEV)
    out = dec.forward(sp, gp)
    rng = np.random.default_rng(seed)
    gi = {k: torch.from_numpy(rng.standard_normal(tuple(v.shape)).astype(np.float32)).to(DEV)
          for k, v in out.items()}
    return dec, sp, gp, gi


def _zeros(dec):
    z = lambda t: torch.zeros(t.shape, dtype=torch.float32, device=DEV)
    return dict(xyz=z(dec.xyz), scaling=z(dec.scaling), offsets=z(dec.offsets), feat=z(dec.feat),
                w1=z(dec.w1), b1=z(dec.b1), w2=z(dec.w2), b2=z(dec.b2))


@pytest.mark.parametrize("first,second", [(("pinhole", 4000, 2), ("lidar", 900, 1)),
                                          (("lidar", 3000, 3), ("pinhole", 500, 0))])
def test_noalloc_decode_backward_matches_the_scratch_entry_point(first, second):
    for step, (kind, n, assets) in enumerate((first, second)):
        _say(f"no-alloc decode backward, call {step}: {kind} {n} anchors + {assets} assets")
        dec, sp, gp, gi = _case(kind, n, assets, seed=31 + step)
        ref = dec.backward(sp, gp, gi, grads=_zeros(dec))
        got = dec.backward(sp, gp, gi, grads=_zeros(dec), noalloc=True)
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(got[k], ref[k]), (step, k, float((got[k] - ref[k]).abs().max()))
        assert float(ref["w2"].abs().max()) > 0 and float(ref["feat"].abs().max()) > 0


def test_noalloc_decode_backward_rejects_inputs_beyond_its_scratch():
    # 64 anchors per block, one camera group of 10 offsets: 17,808 bytes of
    # partials per block; 2000 blocks exceed the 32 MiB array.  The check is
    # on the host: nothing is launched.
    _say("no-alloc decode backward: oversized input is rejected")
    A, K = 2000 * 64, 10
    dec = gs.Decoder(torch.zeros((3, A), device=DEV), torch.ones(A, device=DEV), torch.zeros((3, K, A), device=DEV),
                     torch.zeros((A, 32), dtype=torch.bfloat16, device=DEV),
                     torch.zeros((1, 32, 35), dtype=torch.bfloat16, device=DEV), torch.zeros((1, 32), device=DEV),
                     torch.zeros((1, K * 10, 32), dtype=torch.bfloat16, device=DEV),
                     torch.zeros((1, K * 10), device=DEV), [0, A], lidar=False)
    s = dec._struct()
    nb = ctypes.c_size_t()
    L.check(dec.lib.gs_decode_scratch_size(ctypes.byref(s), ctypes.byref(nb)))
    assert nb.value > L.GS_DECODE_NOALLOC_SCRATCH_BYTES
    pose = torch.tensor([1.0, 0, 0, 0, 0, 1.0, 0, 0, 0, 0, 1.0, 0], device=DEV)
    gi = {k: torch.zeros(v, device=DEV) for k, v in (("mean", (3, A * K)), ("quat", (4, A * K)),
                                                     ("scale", (2, A * K)), ("opacity", (A * K,)),
                                                     ("rgb", (3, A * K)))}
    with pytest.raises(L.GsError) as e:
        dec.backward(pose, pose.view(1, 12), gi, grads=_zeros(dec), noalloc=True)
    assert e.value.status == L.GS_ERR_INVALID_ARG
    # without weight gradients there is no limit
    g = _zeros(dec)
    for k in ("w1", "b1", "w2", "b2"):
        g[k] = None
    dec.backward(pose, pose.view(1, 12), gi, grads=g, noalloc=True)
    torch.cuda.synchronize()
