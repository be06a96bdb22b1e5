"""What the trained initial-density network gains: on a perturbed 64-atom
geometry that was not among its training geometries, the SCF from the
learned guess needs fewer steps than the SCF from the superposition of
atomic densities, starts closer to self-consistency, and converges to the
same energy (the converged SCF, not the network, decides the answer).
Both runs use FP32 cell GEMMs in the filter."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

MODEL = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                     "paper_2607_06848_amd", "weights", "density_c64.npz")
HELD_OUT_SEED = 900


def _say(*a):
    print("[gpu-gain]", *a, flush=True)


def _scf(guess):
    from paper_2607_06848_amd import efe, learned
    from paper_2607_06848_amd import workloads as wl
    w = learned.perturbed_c64(HELD_OUT_SEED)
    ctx = efe.Context(w)
    N = w["nvec"]
    V = torch.from_numpy(wl.random_block(ctx.rows, N, w["v0_seed"])).cuda()
    lam = torch.zeros(N, dtype=torch.float64, device="cuda")
    v0 = torch.from_numpy(wl.random_vector(ctx.rows, 7)).cuda()
    if guess == "learned":
        fb, fac = learned.Model.load(MODEL).apply(ctx)
    else:
        fb, fac = ctx.density_guess(None)
    _say(guess, "fallback", fb, "factor", fac)
    hist = efe.scf_run(ctx, V, lam, v0, w["degree"], tol=1e-5, max_iter=60, prec=efe.EFE_FP32)
    ctx.close()
    _say(guess, len(hist), "steps, E", hist[-1]["E"], "first residual", hist[0]["drho"])
    return fb, hist, len(w["xyz"])


@pytest.fixture(scope="module")
def sad():
    return _scf("sad")


@pytest.fixture(scope="module")
def learned_run():
    if not os.path.exists(MODEL):
        pytest.skip("no trained model in the package")
    return _scf("learned")


def test_superposition_run(sad):
    fb, hist, natoms = sad
    assert fb
    assert abs(hist[-1]["dE"]) / natoms < 1e-5


def test_learned_guess_gains(sad, learned_run):
    _, h0, natoms = sad
    fb, h1, _ = learned_run
    assert not fb, "the network's guess fell back to the superposition"
    assert abs(h1[-1]["dE"]) / natoms < 1e-5
    # same converged answer within the SCF tolerance
    assert abs(h1[-1]["E"] - h0[-1]["E"]) / natoms < 1e-5
    # closer to self-consistency at the start, and fewer SCF steps
    assert h1[0]["drho"] < h0[0]["drho"]
    assert len(h1) < len(h0)
    _say("steps", len(h0), "->", len(h1), "first-step residual", h0[0]["drho"], "->",
         h1[0]["drho"], "dE/atom", abs(h1[-1]["E"] - h0[-1]["E"]) / natoms)
