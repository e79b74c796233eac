"""fbp_reconstruct_noalloc (the entry point for callers that cannot allocate)
against fbp_reconstruct, through the C ABI.

Both run the same kernels; only where the filtered rows live differs (the
library's static workspace against the caller's), so every image must be
bitwise equal.  Two calls in a row go through the one static array, the second
with a smaller input, so a stale first call's rows cannot go unnoticed; one
slice is also held to the FP64 oracle at the FP32 gate.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2109_02174_amd as fbp
from paper_2109_02174_amd import configs, metrics
from paper_2109_02174_amd import phantom as ph

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def _stack(seed, n, N, K, D, dt=1.0, angles=None):
    angles = ph.uniform_angles(K) if angles is None else angles
    out = []
    for i in range(n):
        ell = ph.draw_ellipses(ph.rng_for(seed, i), 8)
        out.append(ph.ellipse_sinogram(ell, N, D, dt, angles))
    return np.stack(out)


def _alone(g, sino, prec):
    return fbp.fbp_reconstruct(g, sino, precision=prec)


def _noalloc(g, sino, prec):
    out = torch.full((sino.shape[0], g.image_size, g.image_size), float("nan"), device=sino.device)
    return fbp.fbp_reconstruct_noalloc(g, sino, out, precision=prec)


def _bitwise(a, b):
    torch.cuda.synchronize()
    return torch.equal(a.view(torch.int32), b.view(torch.int32))


def test_two_calls_in_a_row_match_fbp_reconstruct():
    # first call: four C2-sized slices (8.4 MB of filtered rows); second: one C1 slice
    big = fbp.Geometry(720, 725, 512, 1.0)
    small = fbp.Geometry(180, 183, 128, 1.0)
    s_big = dev(_stack(71, 4, 512, 720, 725))
    c1 = configs.c1_slice()
    s_small = dev(c1.sino[None])
    ref_big = _alone(big, s_big, "fp32")     # makes the plans and taps
    ref_small = _alone(small, s_small, "fp32")
    torch.cuda.synchronize()
    got_big = _noalloc(big, s_big, "fp32")
    got_small = _noalloc(small, s_small, "fp32")
    assert _bitwise(got_big, ref_big)
    assert _bitwise(got_small, ref_small)
    ref = oracle.fbp(c1.sino, c1.N, c1.dt, c1.angles)
    m = metrics.compare(got_small.cpu().numpy()[0].astype(np.float64), ref, c1.value_range)
    assert m["max_abs_rel"] <= 2e-4 and m["rmse_rel"] <= 2e-5, m


@pytest.mark.parametrize("prec", ["bf16", "fp16", "fft"])
def test_other_precisions_match(prec):
    g = fbp.Geometry(90, 101, 70, 1.0)
    s = dev(_stack(72, 2, 70, 90, 101))
    ref = _alone(g, s, prec)
    got = _noalloc(g, s, prec)
    assert _bitwise(got, ref)
    got2 = _noalloc(g, s[:1].contiguous(), prec)
    assert _bitwise(got2, ref[:1])


def test_split_and_stack_shapes_match():
    # non-uniform angles: no quarter-turn pairs, so a single slice may split its
    # angles over the plan's partial sums and 4+ slices take the stack shape
    rng = np.random.default_rng(73)
    ang = np.sort(rng.uniform(0.0, np.pi, 200))
    g = fbp.Geometry(200, 301, 200, 1.0, ang)
    s = dev(_stack(74, 5, 200, 200, 301, angles=ang))
    ref5 = _alone(g, s, "fp32")
    ref1 = _alone(g, s[:1].contiguous(), "fp32")
    got5 = _noalloc(g, s, "fp32")
    got1 = _noalloc(g, s[:1].contiguous(), "fp32")
    assert _bitwise(got5, ref5)
    assert _bitwise(got1, ref1)


def test_fan_beam_matches():
    g = fbp.Geometry(120, 161, 96, 1.0, source_distance=200.0)
    rng = np.random.default_rng(75)
    s = dev(rng.standard_normal((2, 120, 161)))
    ref = _alone(g, s, "fp32")
    got = _noalloc(g, s, "fp32")
    assert _bitwise(got, ref)


def test_refusals_queue_nothing():
    # a geometry with no plan yet, and a precision whose taps were never made
    g = fbp.Geometry(36, 53, 37, 1.0, np.linspace(0.0, 3.0, 36))
    s = dev(np.ones((1, 36, 53)))
    out = torch.zeros((1, 37, 37), device="cuda")
    with pytest.raises(fbp.FbpError) as e:
        fbp.fbp_reconstruct_noalloc(g, s, out)
    assert e.value.status == fbp.FBP_ENOTREADY
    fbp.fbp_reconstruct(g, s, precision="fp32")
    with pytest.raises(fbp.FbpError) as e:
        fbp.fbp_reconstruct_noalloc(g, s, out, precision="bf16")
    assert e.value.status == fbp.FBP_ENOTREADY
    # filtered rows beyond the static workspace: 33 C2 slices need 68.9 MB > 64 MiB
    big = fbp.Geometry(720, 725, 512, 1.0)
    n = fbp.NOALLOC_WORKSPACE_BYTES // (720 * 725 * 4) + 1
    sb = torch.zeros((n, 720, 725), device="cuda")
    ob = torch.zeros((n, 512, 512), device="cuda")
    with pytest.raises(fbp.FbpError) as e:
        fbp.fbp_reconstruct_noalloc(big, sb, ob)
    assert e.value.status == fbp.FBP_EWORKSPACE
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0 and float(ob.abs().max()) == 0.0


def test_replays_of_a_captured_graph_match_eager_calls():
    # the callers this entry point is for: work captured into a HIP graph, where no
    # allocation may happen.  Each replay, with eager work and synchronisations in
    # between, must give the eager images bit for bit.
    g = fbp.Geometry(360, 365, 256, 1.0)
    s = dev(_stack(76, 2, 256, 360, 365))
    ref = _alone(g, s, "fp32")
    out = torch.zeros_like(ref)
    fbp.fbp_reconstruct_noalloc(g, s, out)     # first call on the device outside the capture
    torch.cuda.synchronize()
    assert _bitwise(out, ref)
    side = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        out.zero_()
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=side):
            fbp.fbp_reconstruct_noalloc(g, s, out)
    torch.cuda.synchronize()
    for rep in range(3):
        out.fill_(float(rep + 1))
        _ = _alone(g, s, "fp32")               # eager work between the replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert _bitwise(out, ref), f"replay {rep}"
