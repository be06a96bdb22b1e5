"""Mixed precision: the filter's cell GEMMs in FP32 and BF16 (FP32
accumulation) against the FP64 oracle.  One filter pass is compared element
by element with a bound set by the input rounding of each format; the SCF in
reduced precision must reach the FP64 oracle's converged energy, because the
residual filter's fixed point is exact (the eigen-residual G and the output
term V C_m(Lambda) stay in FP64)."""
import numpy as np
import pytest

from paper_2607_06848_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print("[gpu-mixed]", *a, flush=True)


def _setup(name, **over):
    from oracle import eigen, enrich, fe, psp
    from paper_2607_06848_amd import efe
    w = wl.make(name, **over)
    mesh = fe.Mesh(w["lo"], w["hi"], w["ncell"], w["p"], w["nq"])
    s = enrich.EFESystem(mesh, w)
    X = mesh.quad_coords()
    s.set_potential(sum(psp.v_local(np.linalg.norm(X - R, axis=-1), w["Z"], w["loc_rc"],
                                    w["loc_amp"], w["loc_rg"]) for R in w["xyz"]))
    mask = np.zeros(s.rows)
    mask[s.active()] = 1.0
    V, lam, _ = eigen.rayleigh_ritz(s.apply_H, s.apply_M,
                                    wl.random_block(s.rows, w["nvec"], 5) * mask[:, None], mask)
    b, _, _ = eigen.lanczos_upper_bound(s.apply_H, s.apply_Mtilde, s.apply_Minv_tilde,
                                        wl.random_vector(s.rows, 7) * mask, 20)
    ctx = efe.Context(w)
    ctx.set_potential(ctx.local_potential(), (1 << efe.EFE_FP32) | (1 << efe.EFE_BF16))
    return w, s, V, lam, b, ctx


@pytest.fixture(scope="module", params=["small", "small_cfe"])
def setup(request):
    over = {} if request.param == "small" else dict(enr_lmax=-1, kb_width=0.0)
    out = _setup("small", **over)
    yield out
    out[-1].close()


# unit round-off of the cell GEMM operands (round to nearest: 2^-p for a
# p-bit significand; FP32 p = 24, BF16 p = 8)
UNIT = {"fp32": 2.0 ** -24, "bf16": 2.0 ** -8}


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_filter_reduced_precision(setup, prec):
    """Error of one reduced-precision filter pass relative to the filtered
    residual part M~^-1 Z_m (the only part the cell GEMMs touch: G and
    V C_m(Lambda) stay FP64).

    Error model: every H apply of the recurrence rounds its two cell-GEMM
    operands to unit u, a relative perturbation of at most 2u of each product;
    the filter damps the perturbations of earlier steps as it damps the
    signal, so on plain CFE the output carries about 2u (measured 2.0u in
    FP32, 0.74u in BF16).  With enrichment, (M~^E)^-1 magnifies the rounding
    left in the enrichment rows by up to A (the 2-norm amplification of the
    oracle, ||M^phiphi_II|| / lambda_min(M^ee_II)); measured 0.14 u A on the
    3-atom p = 6 case in FP32.  Bound: u (4 + A / 2), twice the plain term
    and 3.5 times the enriched realization.  BF16 is refused by the library
    beyond its amplification limit (the enriched case)."""
    from oracle import eigen
    from paper_2607_06848_amd import efe
    w, s, V, lam, b, ctx = setup
    m = w["degree"]
    A = ctx.amplification()
    assert A >= s.tilde_condition() * (1 - 1e-9)          # the library's bound covers the oracle's
    p = {"fp32": efe.EFE_FP32, "bf16": efe.EFE_BF16}[prec]
    Vd = torch.from_numpy(V).cuda()
    if prec == "bf16" and A > efe.BF16_MAX_AMPLIFICATION:
        with pytest.raises(efe.EFEError) as e:
            ctx.cheb_filter(Vd, torch.from_numpy(lam).cuda(), m, lam[-1], b, lam[0], prec=p)
        assert e.value.status == -1
        assert np.array_equal(Vd.cpu().numpy(), V)          # refused before any work
        _say(prec, "refused at amplification", A)
        return
    ref = eigen.residual_filter(s.apply_H, s.apply_M, s.apply_Minv_tilde, V, lam, lam[-1], b,
                                lam[0], m)
    base = V * eigen.cheb_scalar(lam, lam[-1], b, lam[0], m)[m][None, :]
    ctx.cheb_filter(Vd, torch.from_numpy(lam).cuda(), m, lam[-1], b, lam[0], prec=p)
    got = Vd.cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref - base).max()
    A2 = s.tilde_condition()
    tol = UNIT[prec] * (4 + A2 / 2)
    _say(prec, "n_enr", s.n_enr, "amplification", A, A2, "error relative to the filtered "
         "residual part", err, "err / u", err / UNIT[prec], "bound", tol)
    assert err < tol


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_scf_reduced_precision_reaches_fp64(prec):
    """The 2-atom SCF with reduced-precision cell GEMMs reaches the FP64
    oracle's converged energy; BF16 is refused when the workload's
    amplification is beyond the library's limit."""
    from oracle import enrich, fe, scf
    from paper_2607_06848_amd import efe
    w = wl.make("eig2")
    mesh = fe.Mesh(w["lo"], w["hi"], w["ncell"], w["p"], w["nq"])
    s = enrich.EFESystem(mesh, w)
    es = scf.Electrostatics(mesh, w["xyz"], w["Zs"], w)
    V0 = wl.random_block(s.rows, w["nvec"], 5)
    v0 = wl.random_vector(s.rows, 7)
    kT = 500 * scf.KB_HA_PER_K
    hist, _ = scf.scf(s, es, V0, v0, w["nvec"], w["degree"], 8.0, kT, tol=1e-9, max_iter=40)
    ctx = efe.Context(w)
    V = torch.from_numpy(V0).cuda()
    lam = torch.zeros(w["nvec"], dtype=torch.float64, device="cuda")
    p = {"fp32": efe.EFE_FP32, "bf16": efe.EFE_BF16}[prec]
    if prec == "bf16" and ctx.amplification() > efe.BF16_MAX_AMPLIFICATION:
        with pytest.raises(efe.EFEError):
            ctx.scf_step(V, lam, torch.from_numpy(v0).cuda(), w["degree"], prec=p, kT=kT)
        _say(prec, "SCF refused at amplification", ctx.amplification())
        ctx.close()
        return
    reps = efe.scf_run(ctx, V, lam, torch.from_numpy(v0).cuda(), w["degree"], tol=1e-9,
                       max_iter=60, prec=p, kT=kT)
    ctx.close()
    dE = abs(reps[-1]["E"] - hist[-1]["E"]) / len(w["xyz"])
    _say(prec, "steps", len(reps), "vs", len(hist), "|E - E_fp64 oracle| per atom", dE,
         "eigenvalue error", np.abs(lam.cpu().numpy() - hist[-1]["lam"]).max())
    assert dE < 1e-5                     # bar of the reduced-precision run; in practice ~1e-9
    # eigenvalues are first order in the density error left by the energy
    # criterion (|dE| < 1e-9 leaves ~1e-5 in rho), on both sides
    assert np.abs(lam.cpu().numpy()[:4] - hist[-1]["lam"][:4]).max() < 1e-4


@pytest.mark.parametrize("which,K,tol", [(0, 4, 1e-15), (1, 4, 1e-6), (2, 32, 2e-2)])
def test_mfma_lane_layout(which, K, tol):
    """The lane mappings the cell kernels assume reproduce A @ B."""
    import ctypes
    from paper_2607_06848_amd import efe
    rng = np.random.default_rng(which)
    A = rng.uniform(-1, 1, (16, K))
    B = rng.uniform(-1, 1, (K, 16))
    Ad, Bd = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    D = torch.zeros((16, 16), dtype=torch.float64, device="cuda")
    st = efe.lib().efe_probe_mfma(which, ctypes.c_void_p(Ad.data_ptr()),
                                  ctypes.c_void_p(Bd.data_ptr()), ctypes.c_void_p(D.data_ptr()))
    assert st == 0
    err = np.abs(D.cpu().numpy() - A @ B).max()
    _say("mfma", which, "max err", err)
    assert err < tol * K


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 2e-2)])
def test_apply_reduced_precision(setup, prec, tol):
    from paper_2607_06848_amd import efe
    w, s, V, lam, b, ctx = setup
    X = wl.random_block(s.rows, 37, 3)
    p = {"fp32": efe.EFE_FP32, "bf16": efe.EFE_BF16}[prec]
    if prec == "bf16" and s.n_enr > 0:
        # the BF16 cell GEMM takes plain CFE systems only
        with pytest.raises(efe.EFEError) as e:
            ctx.apply_H_prec(torch.from_numpy(X).cuda(), p)
        assert e.value.status == -1
        return
    ref = s.apply_H(X)
    got = ctx.apply_H_prec(torch.from_numpy(X).cuda(), p).cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    _say(prec, "apply rel err", err)
    assert err < tol
