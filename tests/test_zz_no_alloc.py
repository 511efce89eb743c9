"""The allocation-free entry point (lt_pipeline_static) against lt_pipeline, through
the C ABI: two calls in a row on one device, the second on a smaller input, each
bit-identical to lt_pipeline's outputs on the same input; a problem larger than the
fixed scratch is refused before any launch."""
import sys

import numpy as np
import pytest

from paper_2504_05808_amd import synth

pytestmark = pytest.mark.gpu

KEYS = ("volume", "shell_count", "max_lt_sq", "mean_lt", "shell_mean_lt", "sphericity", "roundness")


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_05808_amd import lt
    lt.load()
    return torch, lt


def _host(d, t, m):
    out = dict(dist_sq=d.cpu().numpy(), lt_sq=t.cpu().numpy())
    for k in KEYS:
        out[k] = getattr(m, k).cpu().numpy()
    return out


def _outputs(torch, lt, lab, max_label):
    dev = torch.device("cuda:0")
    return (torch.empty(lab.shape, dtype=torch.int32, device=dev),
            torch.empty(lab.shape, dtype=torch.int32, device=dev),
            lt.alloc_measures(max_label + 1, dev))


def test_static_pipeline_two_calls_match_pipeline(gpu):
    torch, lt = gpu
    ctx = lt.Context(0)                    # a context of its own: no scratch grown on it
    big, _ = synth.cfg2()                  # 128^3 int32, 60 objects
    rng = synth.rng_for(41)
    small = synth.random_labels(rng, (37, 45, 70), n_labels=5, p_bg=0.2, blob=4, dtype=np.int32)
    for name, lab in (("128^3 int32", big), ("37x45x70 int32", small)):
        print(f"static pipeline: {name}", flush=True)
        sys.stdout.flush()
        ml = int(lab.max())
        assert lt.pipeline_static_bytes(lab.shape, ml) <= lt.STATIC_SCRATCH_BYTES
        t = torch.from_numpy(lab).cuda()
        got = _host(*lt.pipeline_static(t, ml, out=_outputs(torch, lt, lab, ml), ctx=ctx))
        ctx.sync_status()
        ref = _host(*lt.pipeline(t, ml))
        lt.default_context().sync_status()
        for k in ref:
            np.testing.assert_array_equal(got[k], ref[k], err_msg=f"{name}: {k}")
    ctx.close()


def test_static_pipeline_2d_after_3d(gpu):
    """A 2D call after the 3D ones reuses the same fixed scratch (left dirty)."""
    torch, lt = gpu
    lab, _ = synth.cfg1()
    ml = int(lab.max())
    t = torch.from_numpy(lab).cuda()
    got = _host(*lt.pipeline_static(t, ml, out=_outputs(torch, lt, lab, ml)))
    ref = _host(*lt.pipeline(t, ml))
    lt.default_context().sync_status()
    for k in ref:
        np.testing.assert_array_equal(got[k], ref[k], err_msg=k)


def test_static_pipeline_refuses_large_problem(gpu):
    torch, lt = gpu
    lab = torch.zeros((256, 256, 256), dtype=torch.uint16, device="cuda:0")
    assert lt.pipeline_static_bytes(tuple(lab.shape), 10) > lt.STATIC_SCRATCH_BYTES
    with pytest.raises(lt.LTError) as e:
        lt.pipeline_static(lab, 10, out=_outputs(torch, lt, lab, 10))
    assert e.value.status == 8
