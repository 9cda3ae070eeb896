"""GPU: device memory from a caller allocator (swe_set_allocator).  With
torch's caching allocator, torch counts every byte the library holds and gets
it all back on destroy, and contexts, batches and the server give bitwise the
results of runs on hipMalloc'ed memory."""
import sys
import time

import numpy as np
import pytest
import torch

from paper_2301_12010_amd import inputs, swe

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def single(sc, n, extras):
    s = swe.Solver.from_scenario(sc)
    if extras:
        s.set_outputs([0.5, 1.0])
        s.track_max_depth(True)
        s.set_option(swe.OPT_COMPENSATED, 1)
    s.step(n)
    h, hu, hv, st = s.read()
    out = [h, hu, hv]
    if extras:
        out.append(s.max_depth())
        out.append(s.output(1, wait=True)[0])
    s.close()
    return out, st


def test_torch_allocator_owns_the_memory_and_results_match():
    sc = inputs.dam_break()
    other = inputs.random_wet(96, 40, seed=31)
    n = 60
    ref_x, ref_st = single(sc, n, True)
    ref_plain, _ = single(sc, n, False)
    ref_other, _ = single(other, n, False)
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated()
    sizes = []

    def alloc(nbytes, dev):
        sizes.append(nbytes)
        return torch.cuda.caching_allocator_alloc(nbytes, dev)

    def release(ptr, dev):
        torch.cuda.caching_allocator_delete(ptr)

    swe.set_allocator(alloc, release)
    try:
        say("context with outputs, maximum-depth map and compensated level")
        s = swe.Solver.from_scenario(sc)
        assert torch.cuda.memory_allocated() - m0 >= swe.footprint(sc.params.nx, sc.params.ny)
        s.set_outputs([0.5, 1.0])
        s.track_max_depth(True)
        s.set_option(swe.OPT_COMPENSATED, 1)
        s.step(n)
        h, hu, hv, st = s.read()
        got = [h, hu, hv, s.max_depth(), s.output(1, wait=True)[0]]
        held = torch.cuda.memory_allocated() - m0
        s.close()
        assert torch.cuda.memory_allocated() == m0
        assert len(sizes) == 6  # state, 3 output buffers, map, residual planes
        assert held >= sum(sizes)
        for a, b in zip(got, ref_x):
            assert np.array_equal(a, b)
        assert st["mass"] == ref_st["mass"] and st["t"] == ref_st["t"]

        say("batch")
        bt = swe.Batch()
        i0 = bt.add_scenario(sc, n)
        i1 = bt.add_scenario(other, n)
        bt.run()
        for i, ref in ((i0, ref_plain), (i1, ref_other)):
            for a, b in zip(bt.read(i)[:3], ref):
                assert np.array_equal(a, b)
        assert torch.cuda.memory_allocated() > m0
        bt.close()
        assert torch.cuda.memory_allocated() == m0

        say("server")
        budget = 64 << 20
        sv = swe.Server(mem_budget=budget, max_slots=4)
        assert torch.cuda.memory_allocated() - m0 >= budget
        t = sv.submit_scenario(sc, n)
        t0 = time.time()
        r, state = sv.poll(t)
        while r["status"] == swe.PENDING:
            assert time.time() - t0 < 60, "server did not finish in time"
            time.sleep(0.002)
            r, state = sv.poll(t)
        assert r["status"] == swe.DONE
        for a, b in zip(state, ref_plain):
            assert np.array_equal(a, b)
        sv.close()
        assert torch.cuda.memory_allocated() == m0
    finally:
        swe.set_allocator(None, None)

    say("hipMalloc again")
    again, _ = single(sc, n, False)
    for a, b in zip(again, ref_plain):
        assert np.array_equal(a, b)
    assert torch.cuda.memory_allocated() == m0


def test_failing_allocator_reads_as_out_of_memory():
    sc = inputs.dam_break()
    swe.set_allocator(lambda nbytes, dev: 0, lambda ptr, dev: None)
    try:
        with pytest.raises(swe.SweError) as e:
            swe.Solver.from_scenario(sc)
        assert e.value.code == swe.ENOMEM
    finally:
        swe.set_allocator(None, None)
    s = swe.Solver.from_scenario(sc)
    s.step(5)
    assert s.read()[3]["step"] == 5
    s.close()


def test_misaligned_memory_is_handed_back():
    # memory not aligned to 256 bytes is released at once and the call fails
    # with SWE_EINVAL; no kernel ever sees it
    torch.cuda.synchronize()
    m0 = torch.cuda.memory_allocated()
    released = []

    def alloc(nbytes, dev):
        return torch.cuda.caching_allocator_alloc(nbytes + 256, dev) + 4

    def release(ptr, dev):
        released.append(ptr)
        torch.cuda.caching_allocator_delete(ptr - 4)

    swe.set_allocator(alloc, release)
    try:
        with pytest.raises(swe.SweError) as e:
            swe.Solver.from_scenario(inputs.dam_break())
        assert e.value.code == swe.EINVAL
    finally:
        swe.set_allocator(None, None)
    assert len(released) == 1 and released[0] % 256 == 4
    assert torch.cuda.memory_allocated() == m0
