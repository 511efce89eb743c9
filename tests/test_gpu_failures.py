"""Failure paths on the GPU: injected device-allocation failures (LT_FAULT_INJECT)
at every allocating entry point return LT_E_ALLOC without launching anything and
leave the library usable; the batched form reports device-detected errors per
volume, so one bad volume does not mark the others.  No kernel faults here: the
injected failures stop calls before any launch, and the bad label is an ordinary
input that the kernels flag."""
import numpy as np
import pytest

from oracle import lt_oracle as O
from paper_2504_05808_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_05808_amd import lt
    lt.load()
    return torch, lt


def test_scratch_growth_failure_then_recovery(gpu, monkeypatch):
    torch, lt = gpu
    ctx = lt.Context()
    small = torch.from_numpy(synth.cfg1()[0]).cuda()
    lt.pipeline(small, int(small.max()), ctx=ctx)
    ctx.sync_status()
    lab, _ = synth.cfg2()
    big = torch.from_numpy(lab).cuda()
    monkeypatch.setenv("LT_FAULT_INJECT", "alloc")
    with pytest.raises(lt.LTError) as e:
        lt.pipeline(big, int(lab.max()), ctx=ctx)           # the scratch must grow
    assert e.value.status == 4
    monkeypatch.delenv("LT_FAULT_INJECT")
    d, t, m = lt.pipeline(big, int(lab.max()), ctx=ctx)
    ctx.sync_status()
    ref = O.measure(lab)
    np.testing.assert_array_equal(t.cpu().numpy(), ref["lt_sq"])
    ctx.close()


def test_context_creation_fails_part_way(gpu, monkeypatch):
    torch, lt = gpu
    for n_ok in (0, 1, 2):
        monkeypatch.setenv("LT_FAULT_INJECT", f"alloc:{n_ok}")
        with pytest.raises(lt.LTError) as e:
            lt.Context()
        assert e.value.status == 4
        monkeypatch.delenv("LT_FAULT_INJECT")
    ctx = lt.Context()                                    # usable again
    lab, _ = synth.cfg1()
    t = torch.from_numpy(lab).cuda()
    _, ltsq, _ = lt.pipeline(t, int(lab.max()), ctx=ctx)
    ctx.sync_status()
    np.testing.assert_array_equal(ltsq.cpu().numpy(), O.measure(lab, per_object=False)["lt_sq"])
    ctx.close()


def test_network_and_batch_creation_failures(gpu, monkeypatch):
    torch, lt = gpu
    ctx = lt.default_context()
    monkeypatch.setenv("LT_FAULT_INJECT", "alloc")
    with pytest.raises(lt.LTError) as e:
        lt.MLP(seed=1)
    assert e.value.status == 4
    vols = [(torch.from_numpy(synth.cfg1()[0]).cuda(), 20)]
    with pytest.raises(lt.LTError) as e:
        lt.Batch(vols)
    assert e.value.status == 4
    monkeypatch.delenv("LT_FAULT_INJECT")
    b = lt.Batch(vols)
    b.run()
    assert b.status() == [0]
    b.close()


def test_batch_reports_the_bad_volume_only(gpu):
    torch, lt = gpu
    rng = synth.rng_for(4242)
    labs = [synth.random_labels(rng, s, n_labels=5, p_bg=0.2, blob=4, dtype=np.uint16)
            for s in ((20, 30, 40), (24, 28, 32), (16, 50, 20))]
    bad = labs[1].copy()
    bad[3, 4, 5] = 9                                      # above this volume's max_label 5
    vols = [(torch.from_numpy(labs[0]).cuda(), 5), (torch.from_numpy(bad).cuda(), 5),
            (torch.from_numpy(labs[2]).cuda(), 5)]
    b = lt.Batch(vols)
    for _ in range(2):                                    # statuses are re-read and cleared per call
        b.run()
        assert b.status() == [0, 6, 0]
    lt.default_context().sync_status()                    # the context's own word stays clear
    for i in (0, 2):
        ref = O.measure(labs[i], max_label=5, per_object=False)
        d, t, m = b.outputs[i]
        np.testing.assert_array_equal(t.cpu().numpy(), ref["lt_sq"])
        np.testing.assert_array_equal(m.volume.cpu().numpy().astype(np.int64), ref["volume"])
    b.close()
