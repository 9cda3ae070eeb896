"""swe_run_noalloc (the allocation-free run on caller device arrays) against
swe_create / swe_step / swe_read on the same scenario, through the C ABI.

Both run the same conversions and stage kernels, so the states and the
diagnostics are compared bitwise; two calls in a row (the second on a
smaller grid, with FIXED sides) check that the shared working array keeps
nothing from the earlier call that matters."""
import sys

import numpy as np
import pytest

from paper_2301_12010_amd import inputs, swe

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def context_run(sc, nsteps):
    s = swe.Solver.from_scenario(sc)
    s.set_option(swe.OPT_GRAPH_STEPS, 0)
    s.step(nsteps)
    out = s.read()
    s.close()
    return out


def noalloc_run(sc, nsteps, stream=None, stats=True):
    import torch
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in sc.fields()]
    torch.cuda.synchronize()
    st = swe.run_noalloc(sc.params, *dev, nsteps, stream=stream, stats=stats)
    torch.cuda.synchronize()
    return dev[2].cpu().numpy(), dev[3].cpu().numpy(), dev[4].cpu().numpy(), st


def assert_same(a, b, label):
    for x, y, name in zip(a[:3], b[:3], ("h", "hu", "hv")):
        assert np.array_equal(x, y), (label, name, float(np.abs(x - y).max()))
    for k in ("t", "step", "mass", "dt", "alpha_x", "alpha_y", "runup", "status"):
        assert a[3][k] == b[3][k], (label, k, a[3][k], b[3][k])
    # the clamped mass is summed with FP64 atomics in the order blocks finish,
    # so two runs of the same kernels agree to rounding, not bitwise
    assert abs(a[3]["clamp_mass"] - b[3]["clamp_mass"]) <= 1e-12 * max(abs(b[3]["clamp_mass"]), 1e-300)


def test_noalloc_equals_context_on_two_calls_in_a_row():
    big = inputs.mitigation_coast(384, 320, 2.0, seed=1004)        # reflective, wet/dry coast
    small = inputs.steady_slope(nx=130, ny=37, perturb=0.05)       # FIXED west/east sides
    for sc, n in ((big, 40), (small, 25)):
        say(f"case {sc.name} {sc.params.nx}x{sc.params.ny} steps={n}")
        ref = context_run(sc, n)
        got = noalloc_run(sc, n)
        assert_same(got, ref, sc.name)
        assert got[3]["step"] == n and got[3]["status"] == swe.OK


def test_noalloc_asynchronous_on_a_stream_then_stats():
    import torch
    sc = inputs.random_wet(100, 70, seed=5, dry_fraction=0.05)
    ref = context_run(sc, 12)
    stream = torch.cuda.Stream()
    got = noalloc_run(sc, 12, stream=stream, stats=False)
    assert got[3] is None
    for x, y in zip(got[:3], ref[:3]):
        assert np.array_equal(x, y)


def test_noalloc_rejects_what_does_not_fit_or_is_not_on_the_device():
    import torch
    sc = inputs.random_wet(40, 30, seed=6)
    dev = [torch.from_numpy(a).cuda() for a in sc.fields()]
    with pytest.raises(swe.SweError) as ei:
        swe.run_noalloc(sc.params, sc.b, *dev[1:], 3)  # host bed array
    assert ei.value.code == swe.EINVAL
    p = inputs.Params(1600, 1200, 1.0, 1.0)  # 1.92 M cells: beyond the fixed array
    assert swe.footprint(1600, 1200) > swe.NOALLOC_MAX_BYTES
    big = [torch.zeros((1200, 1600), device="cuda") for _ in range(5)]
    with pytest.raises(swe.SweError) as ei:
        swe.run_noalloc(p, *big, 1)
    assert ei.value.code == swe.EINVAL
    bad = [t.clone() for t in dev]
    bad[2][3, 3] = float("nan")
    with pytest.raises(swe.SweError) as ei:
        swe.run_noalloc(sc.params, *bad, 2)
    assert ei.value.code == swe.EINVAL
    # still fine afterwards
    got = noalloc_run(sc, 3)
    assert_same(got, context_run(sc, 3), "after errors")
