"""flame_step_noalloc (the allocation-free entry point) against flame_step on
a plan in its default configuration, through the C ABI, on consecutive calls
that share the library's static scratch: 2048 x 4096, then smaller grids."""

import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth
from flame_testlib import oracle_params, rel_l2
from paper_0911_2889_amd import FlameSim, native

pytestmark = pytest.mark.gpu


def _noalloc(desc, state, n, nsteps):
    lib = native.load()
    stream = torch.cuda.current_stream()
    native.check(lib.flame_step_noalloc(ctypes.byref(desc), ctypes.c_void_p(state.data_ptr()), int(n), int(nsteps),
                                        ctypes.c_void_p(stream.cuda_stream)))


def _both_paths(name, steps, n0=0):
    """(no-alloc half spectrum, plan half spectrum, initial half spectrum, workload)."""
    w = synth.WORKLOADS[name]
    half = synth.workload_spectrum(w)
    print(f"no-alloc case {name}: {steps} steps from step index {n0}", flush=True)
    sim = FlameSim(w.n1, w.n2, gamma=w.gamma, theta_pi=w.theta_pi, t0=w.t0, dt=w.dt, device="cuda:0")
    sim.set_spectrum(half, n=n0)
    state0 = sim.states[0].clone()
    sim.step(steps)
    ref = sim.spectrum().cpu().numpy()
    st = state0.clone()
    _noalloc(sim.descs[0], st, n0, steps)
    # read the result back through the plan's canonical layout
    sim.states[0].copy_(st)
    sim.state_modified(n0 + steps)
    got = sim.spectrum().cpu().numpy()
    torch.cuda.synchronize()
    return got, ref, half, w


def test_noalloc_matches_flame_step_on_consecutive_calls():
    # the benchmark's grid and launch configuration first
    got, ref, _, _ = _both_paths("flame2048x4096", 5)
    e_big = rel_l2(got, ref)
    # then smaller grids, reusing the scratch the first call left behind
    got2, ref2, half2, w2 = _both_paths("flame512x1024", 20, n0=7)
    e_mid = rel_l2(got2, ref2)
    got3, ref3, half3, w3 = _both_paths("flame64x128", 30)
    e_small = rel_l2(got3, ref3)
    print(f"no-alloc vs flame_step: {e_big:.2e} (2048x4096), {e_mid:.2e} (512x1024), {e_small:.2e} (64x128); "
          f"bitwise: {np.array_equal(got, ref)}, {np.array_equal(got2, ref2)}, {np.array_equal(got3, ref3)}")
    assert e_big <= 1e-6 and e_mid <= 1e-6 and e_small <= 1e-6
    # and against the FP64 oracle on the smaller grids
    for got_h, half, w, steps, n0 in ((got2, half2, w2, 20, 7), (got3, half3, w3, 30, 0)):
        p = oracle_params(w)
        full = oracle.run(oracle.half_to_full(half.astype(np.complex128), w.n1, w.n2), p, steps, n_start=n0)
        err = rel_l2(got_h, oracle.full_to_half(full, w.n1, w.n2))
        print(f"no-alloc vs oracle, {w.name}: {err:.2e}")
        assert err <= 1e-5


def test_noalloc_rejects_what_it_cannot_run():
    st = torch.zeros(64 * 128 // 8, dtype=torch.complex64, device="cuda:0")
    lib = native.load()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    too_big = native.make_desc(4096, 4096)
    assert lib.flame_step_noalloc(ctypes.byref(too_big), ctypes.c_void_p(st.data_ptr()), 0, 1, stream) == \
        native.FLAME_ERR_WORKSPACE_TOO_SMALL
    heun = native.make_desc(64, 128, integrator=1)
    assert lib.flame_step_noalloc(ctypes.byref(heun), ctypes.c_void_p(st.data_ptr()), 0, 1, stream) == \
        native.FLAME_ERR_INVALID_ARG
    ok = native.make_desc(64, 128)
    assert lib.flame_step_noalloc(ctypes.byref(ok), ctypes.c_void_p(st.data_ptr()), 0, -1, stream) == \
        native.FLAME_ERR_INVALID_ARG
