"""Batch invariance of the whole-frame kernels.

A task carries up to max_batch frames of one size and every layer runs once
for all of them; the kernels index their pixel tiles across the images of
the batch.  At 720p (N=128, M=192) and 1080p (N=192, M=320) every layer takes
its whole-frame kernel (split-FP32, bf16 or e4m3 GDN layers with the LDS
weight and gamma staging, the halo-tile output layer), so these sizes check
the image-index arithmetic that the small-size batch tests (split-K kernels)
never reach.  For each layer, a launch over n frames must give exactly the
bits of n single-frame launches on the same inputs, in all three operand
forms; and the pipelined codec with tasks of n frames must give the same
bitstreams and pixels as tasks of one frame.
"""
import numpy as np
import pytest

import synth
from gpu_util import layer_out_shape, make_codec

pytestmark = pytest.mark.gpu

CASES = [(0, 128, 192, 720, 1280, 3), (1, 128, 192, 720, 1280, 3), (2, 128, 192, 720, 1280, 3),
         (0, 192, 320, 1080, 1920, 4), (1, 192, 320, 1080, 1920, 4), (2, 192, 320, 1080, 1920, 4)]

# layer, input key, output dtype key, aux dtype key
CHAIN = [("GA0", "x", "act", None), ("GA1", "GA0", "act", None), ("GA2", "GA1", "act", None),
         ("GA3", "GA2", "f32", "i8"), ("HA0", "GA3", "f32", None), ("HA1", "HA0", "f32", None),
         ("HA2", "HA1", "f32", "i8"), ("HS0", "HA2:aux", "f32", None), ("HS1", "HS0", "f32", None),
         ("HS2", "HS1", "u8", "f32"), ("GS0", "GA3:aux", "act", None), ("GS1", "GS0", "act", None),
         ("GS2", "GS1", "act_gs2", None), ("GS3", "GS2", "img", "pre")]


@pytest.mark.parametrize("prec,N,M,H,W,n", CASES, ids=lambda v: str(v))
def test_layers_batched_equal_single(prec, N, M, H, W, n):
    import torch
    assert torch.cuda.is_available()
    c, _ = make_codec(1, N, M, gamma="dense", precision=prec, max_h=H, max_w=W, max_in_flight=1, max_batch=n)
    act = {0: torch.float32, 1: torch.bfloat16, 2: torch.uint8}[prec]
    # (the e4m3 form's GS2 stores bf16 for its output layer's bf16 operands)
    dt = {"act": act, "act_gs2": torch.bfloat16 if prec == 2 else act, "f32": torch.float32, "u8": torch.uint8,
          "i8": torch.int8}
    Hp, Wp = 64 * -(-H // 64), 64 * -(-W // 64)

    def alloc(L, key, k):
        if key == "img":
            return torch.empty((k, 3, H, W), device="cuda")
        if key == "pre":
            return torch.empty((k, 3, Hp, Wp), device="cuda")
        return torch.empty((k,) + layer_out_shape(L, H, W, N, M), device="cuda", dtype=dt[key])

    x = torch.from_numpy(np.stack([synth.frame_sinusoid(H, W, t=t, stream=3) for t in range(n)])).cuda()
    outs = {"x": x}
    for L, src, okey, akey in CHAIN:
        inp = outs[src]
        o = alloc(L, okey, n)
        a = None if akey is None else alloc(L, akey, n)
        c.run_layer(L, n, H, W, inp, o, a)
        outs[L], outs[L + ":aux"] = o, a
        for i in range(n):
            o1 = alloc(L, okey, 1)
            a1 = None if akey is None else alloc(L, akey, 1)
            c.run_layer(L, 1, H, W, inp[i:i + 1].contiguous(), o1, a1)
            assert torch.equal(o1[0], o[i]), f"{L}: image {i} of a batch of {n} differs from the image alone"
            if a is not None:
                assert torch.equal(a1[0], a[i]), f"{L} (second output): image {i} of {n} differs"
    c.close()


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_codec_tasks_of_four_equal_single_frames_1080p(prec):
    """The precision-form workload: 1080p frames, N=192 M=320, tasks of 4 frames."""
    import torch
    H, W, N, M = 1080, 1920, 192, 320
    c1, _ = make_codec(1, N, M, precision=prec, max_h=H, max_w=W, y_slices=8, entropy_threads=8, max_in_flight=2)
    c4, _ = make_codec(1, N, M, precision=prec, max_h=H, max_w=W, y_slices=8, entropy_threads=8, max_in_flight=2,
                       max_batch=4)
    xs = torch.from_numpy(np.stack([synth.frame_sinusoid(H, W, t=t, stream=4) for t in range(6)])).cuda()
    b1, b4 = c1.encode(xs), c4.encode(xs)
    assert b1 == b4
    o1 = torch.empty_like(xs)
    o4 = torch.empty_like(xs)
    c1.decode(b1, o1)
    c4.decode(b4, o4)
    assert torch.equal(o1, o4)
    c1.close()
    c4.close()
