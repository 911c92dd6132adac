"""Adjoint of the HIP step and of the area functional against the FP64 oracle."""

import numpy as np
import pytest

import oracle
import synth
from flame_testlib import rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def to_internal(half, n1, n2):
    """Canonical half array -> state layout S[m][s], s = k1 + N1/4 (test-side marshalling)."""
    s = np.zeros((n2 // 4, n1 // 2), dtype=np.complex64)
    s[:, 1:] = np.asarray(half).T
    return torch.from_numpy(s.reshape(-1)).to("cuda")


def from_internal(t, n1, n2):
    s = t.cpu().numpy().reshape(n2 // 4, n1 // 2)
    return s[:, 1:].T.copy()


def spectrum(n1, n2, seed, amp):
    w = synth.Workload("a", n1, n2, 1, 0.1, "all", amp, -1.0, seed)
    return synth.workload_spectrum(w)


def make(n1, n2, t0, dt, **kw):
    from paper_0911_2889_amd import FlameSim
    return FlameSim(n1, n2, t0=t0, dt=dt, **kw)


@pytest.mark.parametrize("n1,n2", [(64, 128), (128, 64), (256, 512), (32, 4096), (2048, 64)])
def test_adjoint_step_matches_oracle(n1, n2):
    t0, dt, n = 5.0, 0.2, 3
    state = spectrum(n1, n2, 11 + n1, 0.3)
    lam = spectrum(n1, n2, 12 + n2, 1.0)
    sim = make(n1, n2, t0, dt)
    st = to_internal(state, n1, n2)
    li = to_internal(lam, n1, n2)
    lo = torch.zeros_like(li)
    sim.adjoint_step(n, st, li, lo)
    got = from_internal(lo, n1, n2)
    p = oracle.Params(n1, n2, t0=t0, dt=dt)
    sf = oracle.half_to_full(state.astype(np.complex128), n1, n2)
    lf = oracle.half_to_full(lam.astype(np.complex128), n1, n2)
    ref = oracle.full_to_half(oracle.step_adjoint(sf, lf, p, n), n1, n2)
    linear = oracle.full_to_half(np.exp(oracle.growth_exponent(p, n)) * lf * oracle.box_mask(n1, n2), n1, n2)
    assert rel_l2(ref, linear) > 1e-3  # the quadratic term's adjoint matters here
    assert rel_l2(got, ref) < 1e-5
    # in place (lam_out == lam_in) gives the same bits
    sim.adjoint_step(n, st, li, li)
    assert np.array_equal(from_internal(li, n1, n2), got)


@pytest.mark.parametrize("n1,n2", [(64, 128), (256, 256), (1024, 64)])
def test_area_gradient_matches_oracle(n1, n2):
    t0, n = 3.0, 4
    state = spectrum(n1, n2, 21 + n1, 0.5)
    sim = make(n1, n2, t0, 0.1)
    lo = sim.new_cotangent()
    sim.area_gradient(n, to_internal(state, n1, n2), lo)
    got = from_internal(lo, n1, n2)
    p = oracle.Params(n1, n2, t0=t0, dt=0.1)
    ref = oracle.full_to_half(oracle.area_gradient(oracle.half_to_full(state.astype(np.complex128), n1, n2), p, n),
                              n1, n2)
    assert rel_l2(got, ref) < 1e-5


@pytest.mark.parametrize("n1,n2", [(64, 128), (256, 512)])
def test_diagnostics_seed_is_the_area_gradient(n1, n2):
    """flame_diagnostics with a seed buffer writes the area gradient at the
    current state and step index (the oracle's, and area_gradient's bits),
    besides the averages; after it the step rebuilds its intermediates."""
    t0, dt, steps = 3.0, 0.1, 5
    half = spectrum(n1, n2, 31 + n1, 0.3)
    sim = make(n1, n2, t0, dt)
    sim.set_spectrum(half)
    sim.step(steps)
    seed = sim.new_cotangent()
    d = sim.diagnostics(dJ_dstate=seed)
    assert d["finite"]
    lo = sim.new_cotangent()
    sim.area_gradient(steps, sim.states[0].clone(), lo)
    assert torch.equal(seed, lo)
    state = oracle.half_to_full(sim.spectrum().cpu().numpy().astype(np.complex128), n1, n2)
    p = oracle.Params(n1, n2, t0=t0, dt=dt)
    ref = oracle.full_to_half(oracle.area_gradient(state, p, steps), n1, n2)
    assert rel_l2(from_internal(seed, n1, n2), ref) < 1e-5
    # the intermediates are rebuilt: the next steps equal an undisturbed run's
    ref_sim = make(n1, n2, t0, dt)
    ref_sim.set_spectrum(half)
    ref_sim.step(steps + 3)
    sim.step(3)
    assert np.array_equal(sim.spectrum().cpu().numpy(), ref_sim.spectrum().cpu().numpy())


def test_state_modified_marks_one_flame_or_all():
    from paper_0911_2889_amd import FlameEnsemble, native
    descs = [dict(n1=64, n2=128, t0=3.0, dt=0.1), dict(n1=128, n2=256, t0=3.0, dt=0.1)]
    halves = [spectrum(d["n1"], d["n2"], 40 + i, 0.2) for i, d in enumerate(descs)]
    ens = FlameEnsemble(descs)
    for f, h in enumerate(halves):
        ens.set_spectrum(h, flame=f)
    ens.step(4)
    saved = ens.states[1].clone()
    ens.step(2)
    ens.states[1].copy_(saved)  # restore flame 1 only
    assert ens.lib.flame_state_modified(ens.plan, 2, 6) == native.FLAME_ERR_INVALID_ARG  # no flame 2
    ens.state_modified(4, flame=1)  # one step index for the plan: flame 0 goes on from 6 as if at 4
    ens.step(2)
    ref = FlameEnsemble(descs[1:])
    ref.set_spectrum(halves[1], flame=0)
    ref.step(6)
    assert np.array_equal(ens.spectrum(1).cpu().numpy(), ref.spectrum(0).cpu().numpy())
    ens.state_modified(6, flame=-1)
    ens.step(1)
    assert ens.step_index == 7


def test_synthesize_matches_get_state():
    n1, n2 = 128, 256
    half = spectrum(n1, n2, 5, 0.1)
    sim = make(n1, n2, 200.0, 0.25)
    sim.set_spectrum(half)
    a = sim.phi()
    b = sim.synthesize(sim.states[0])
    assert torch.equal(a, b)


@pytest.mark.parametrize("n1,n2,nsteps,every", [(64, 128, 20, 7), (128, 128, 12, 12), (32, 64, 9, 1)])
def test_checkpointed_gradient_matches_oracle(n1, n2, nsteps, every):
    from paper_0911_2889_amd import flame_area
    t0, dt = 3.0, 0.2
    phi0 = synth.physical_noise(n1, n2, seed=n1 + nsteps, kind="normal", scale=0.3)
    sim = make(n1, n2, t0, dt)
    x = torch.from_numpy(phi0).to("cuda").requires_grad_(True)
    J = flame_area(x, sim, nsteps, checkpoint_every=every)
    J.backward()
    got = x.grad.cpu().numpy().astype(np.float64)
    p = oracle.Params(n1, n2, t0=t0, dt=dt)
    full0 = oracle.project(phi0.astype(np.float64))
    jref, lam = oracle.trajectory_gradient(full0, p, nsteps)
    ref = oracle.synthesize(lam).real
    assert abs(J.item() - jref) < 1e-5 * abs(jref)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-5


@pytest.mark.parametrize("n1,n2", [(256, 512), (1024, 128), (128, 2048)])
def test_adjoint_step_on_both_grids_matches_oracle(n1, n2):
    """The adjoint step on the 3*N1/4-row product grid (the transpose of the
    step the product grid takes) and on N1 rows, against the oracle's
    transposed step."""
    t0, dt, n = 5.0, 0.2, 2
    state = spectrum(n1, n2, 31 + n1, 0.3)
    lam = spectrum(n1, n2, 32 + n2, 1.0)
    p = oracle.Params(n1, n2, t0=t0, dt=dt)
    sf = oracle.half_to_full(state.astype(np.complex128), n1, n2)
    lf = oracle.half_to_full(lam.astype(np.complex128), n1, n2)
    ref = oracle.full_to_half(oracle.step_adjoint(sf, lf, p, n), n1, n2)
    got = {}
    for product in (True, False):
        sim = make(n1, n2, t0, dt)
        sim.set_product_grid(n1, n2, product)
        lo = sim.new_cotangent()
        sim.adjoint_step(n, to_internal(state, n1, n2), to_internal(lam, n1, n2), lo)
        got[product] = from_internal(lo, n1, n2)
        assert rel_l2(got[product], ref) < 1e-5, product
    assert rel_l2(got[True], got[False]) < 2e-6
