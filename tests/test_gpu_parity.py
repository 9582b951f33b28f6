"""HIP path vs the FP64 oracle, through the C ABI (MI355X only).

Tolerances (FP64 path): max_ij |dH_ij| / max_ij |H_ij| <= 1e-10, max |dS| <= 1e-10,
|dE| <= 1e-10 (1 + |E|).  These hold while the smallest relative singular-value
gap at a truncation cut stays well above the rounding level; every workload
below has its gap printed by the oracle (>= 1e-7).
"""
import os

import numpy as np
import pytest

import paper_2404_10223_amd as T
import tnqe_synth as synth
from oracle import fock, gep
from oracle.subspace import subspace as oracle_subspace

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
RTOL = 1e-10


@pytest.fixture(scope="module")
def ctx():
    c = T.Context(0)
    yield c
    c.close()


def _assert_pencil(H, S, E, Ho, So, Eo, tol=RTOL, elementwise=False):
    dH = np.abs(H - Ho).max() / np.abs(Ho).max()
    dS = np.abs(S - So).max()
    print(f"dH_rel={dH:.2e} dS={dS:.2e} dE={abs(E - Eo):.2e}", flush=True)
    assert dH <= tol
    assert dS <= tol
    assert abs(E - Eo) <= tol * (1 + abs(Eo))
    if elementwise:
        # every element to the tolerance relative to itself (the off-diagonal
        # elements are orders of magnitude below the diagonal)
        assert np.all(np.abs(H - Ho) <= tol * np.abs(Ho)), np.max(np.abs(H - Ho) / np.abs(Ho))
        assert np.all(np.abs(S - So) <= tol * np.abs(So)), np.max(np.abs(S - So) / np.abs(So))
    np.testing.assert_array_equal(H, H.T)
    np.testing.assert_array_equal(S, S.T)


def _assert_report(rep, Ho, So):
    """cond(S), lambda_min(S), kappa_1 and the dropped count of the library
    against the oracle's eigensolver on the oracle's pencil (App. A2)."""
    o = gep.solve_projection(Ho, So)
    print(f"cond_S={rep['cond_S']:.6e} ({o['cond_S']:.6e}) lambda_min={rep['lambda_min_S']:.6e} "
          f"({o['lam_min']:.6e}) kappa1={rep['kappa1']:.6e} ({o['kappa1']:.6e})", flush=True)
    assert rep["n_dropped"] == o["n_dropped"]
    assert abs(rep["lambda_min_S"] - o["lam_min"]) <= 1e-10 * max(1.0, abs(o["lam_min"]))
    assert abs(rep["cond_S"] - o["cond_S"]) <= 1e-8 * o["cond_S"]
    assert abs(rep["kappa1"] - o["kappa1"]) <= 1e-8 * o["kappa1"]


@pytest.mark.parametrize("k", [1, 2, 3])
def test_config_parity_fp64(ctx, k):
    prob = synth.make_config(k)
    g = np.load(os.path.join(GOLD, f"oracle_config{k}.npz"))
    H, S, E, c, rep = ctx.subspace(prob, chi=prob.chi)
    _assert_pencil(H, S, E, g["H"], g["S"], float(g["E"]), elementwise=True)
    _assert_report(rep, g["H"], g["S"])
    assert abs(rep["max_discarded_weight_sum"] - float(g["max_discarded"])) < 1e-10
    np.testing.assert_allclose(np.diag(S), 1.0, atol=1e-12)
    assert abs(c @ S @ c - 1.0) < 1e-10


@pytest.mark.parametrize("k", [1, 2, 3])
def test_workspace_path(ctx, k):
    """tnqe_subspace with a caller-allocated device workspace (torch): every
    device buffer of the call lies in it; same results as the pooled path."""
    import torch
    prob = synth.make_config(k)
    g = np.load(os.path.join(GOLD, f"oracle_config{k}.npz"))
    n = ctx.workspace_size(prob, chi=prob.chi)
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    H, S, E, c, rep = ctx.subspace(prob, chi=prob.chi, workspace=ws)
    print(f"workspace {n / 2 ** 20:.1f} MiB, used {rep['ws_peak_bytes'] / 2 ** 20:.1f} MiB", flush=True)
    _assert_pencil(H, S, E, g["H"], g["S"], float(g["E"]), elementwise=True)
    assert 0 < rep["ws_peak_bytes"] <= n
    # a workspace below what the call needs is refused cleanly, and the
    # context goes on working (the environment sweep fills what it is given
    # with pair batches, so only far smaller sizes fail)
    small = torch.empty(4096, dtype=torch.uint8, device="cuda")
    with pytest.raises(T.TnqeError) as e:
        ctx.subspace(prob, chi=prob.chi, workspace=small)
    assert e.value.status == -6
    H2, S2, E2, _, _ = ctx.subspace(prob, chi=prob.chi, workspace=ws)
    np.testing.assert_array_equal(H2, H)
    np.testing.assert_array_equal(S2, S)


def test_workspace_smaller_than_common_layout(ctx):
    """A workspace that holds the gate phase but not one pair of the common
    environment layout: every pair then runs alone in its own layout."""
    import torch
    prob = synth.make_config(3)
    g = np.load(os.path.join(GOLD, "oracle_config3.npz"))
    big = torch.empty(ctx.workspace_size(prob, chi=prob.chi), dtype=torch.uint8, device="cuda")
    _, _, _, _, rep = ctx.subspace(prob, chi=prob.chi, workspace=big)
    lo, hi = 1, int(rep["ws_peak_bytes"])
    got = None
    # the smallest workspace (to 1 %) that still works: it takes the own-layout route
    while hi - lo > hi // 100:
        mid = (lo + hi) // 2
        try:
            got = ctx.subspace(prob, chi=prob.chi, workspace=big[:mid])
            hi = mid
        except T.TnqeError as e:
            assert e.status == -6
            lo = mid
    H, S, E, c, rep2 = ctx.subspace(prob, chi=prob.chi, workspace=big[:hi])
    print(f"smallest workspace {hi / 2 ** 20:.1f} MiB of {rep['ws_peak_bytes'] / 2 ** 20:.1f}", flush=True)
    _assert_pencil(H, S, E, g["H"], g["S"], float(g["E"]), elementwise=True)


def test_device_gep_hand_solved(ctx):
    """The device eigensolver on pencils solved by hand (App. A2: kappa_1,
    thresholding of S)."""
    r = ctx.debug_gep(np.array([[0.0, 1.0], [1.0, 0.0]]), np.array([[1.0, 0.5], [0.5, 1.0]]))
    assert r["status"] == 0 and abs(r["E"] + 2.0) < 1e-14
    assert abs(abs(r["c"][0]) - 1.0) < 1e-13 and abs(r["c"][0] + r["c"][1]) < 1e-13
    assert abs(r["kappa1"] - 2.0 / np.sqrt(5.0)) < 1e-13
    assert abs(r["cond_S"] - 3.0) < 1e-12 and abs(r["lambda_min"] - 0.5) < 1e-14 and r["n_dropped"] == 0
    r = ctx.debug_gep(np.diag([-8.0, 1.0, 5.0]), np.diag([4.0, 1e-3, 1e-14]))
    assert r["n_dropped"] == 1 and abs(r["E"] + 2.0) < 1e-14
    np.testing.assert_allclose(np.abs(r["c"]), [0.5, 0.0, 0.0], atol=1e-15)
    assert abs(r["kappa1"] - 0.25 / np.sqrt(5.0)) < 1e-15 and abs(r["cond_S"] - 4e3) < 1e-9
    assert r["lambda_min"] == 1e-14
    r = ctx.debug_gep(np.diag([-1.0, 2.0]), np.diag([1.0, -1e-9]))
    assert r["n_dropped"] == 1 and r["lambda_min"] == -1e-9 and abs(r["E"] + 1.0) < 1e-15
    # random pencils against the oracle, up to M = 32
    rng = np.random.default_rng(11)
    for M in (3, 16, 32):
        A = rng.normal(size=(M, M))
        S = A @ A.T / M + np.eye(M)
        H = rng.normal(size=(M, M))
        H = H + H.T
        r = ctx.debug_gep(H, S)
        o = gep.solve_projection(H, S)
        assert abs(r["E"] - o["E"]) < 1e-12 * max(1.0, abs(o["E"]))
        assert abs(r["kappa1"] - o["kappa1"]) < 1e-10 * o["kappa1"]
        assert abs(r["cond_S"] - o["cond_S"]) < 1e-10 * o["cond_S"]


def test_renormalized_truncation(ctx):
    """renormalize = 1 (the kept part rescaled after every cut) against the
    oracle with the same option."""
    prob = synth.make_config(2)
    Ho, So, Eo, co, rep_o = oracle_subspace(prob, renormalize=True)
    H, S, E, c, rep = ctx.subspace(prob, chi=prob.chi, renormalize=True)
    _assert_pencil(H, S, E, Ho, So, Eo, elementwise=True)
    H0, S0, _, _, _ = ctx.subspace(prob, chi=prob.chi)
    assert np.abs(S - S0).max() > 1e-6          # the option changes the result


@pytest.mark.parametrize("rot", ["perm", "identity"])
@pytest.mark.parametrize("k", [2, 3])
def test_variant_workloads_parity_fp64(ctx, k, rot):
    """Fermionic-swap networks (orbital permutations, TNQE-F; det = -1 cases
    take the parity gate) and no rotations at all (LC-MPS) on the same path."""
    prob = synth.make_config(k, rot)
    g = np.load(os.path.join(GOLD, f"oracle_{prob.name}.npz"))
    print(prob.name, "oracle min_rel_gap", float(g["min_rel_gap"]), flush=True)
    H, S, E, c, rep = ctx.subspace(prob, chi=prob.chi)
    _assert_pencil(H, S, E, g["H"], g["S"], float(g["E"]), elementwise=True)
    assert abs(rep["max_discarded_weight_sum"] - float(g["max_discarded"])) < 1e-10
    np.testing.assert_allclose(np.diag(S), 1.0, atol=1e-12)


def test_lossless_matches_brute_force(ctx):
    prob = synth.make_config(1)
    H, S, E, c, rep = ctx.subspace(prob, chi=prob.chi, chi_cap_override=10 ** 6)
    Ho, So, Eo, co, _ = oracle_subspace(prob, chi_cap=10 ** 6)
    _assert_pencil(H, S, E, Ho, So, Eo, 1e-12)
    # against the 4^N Fock space directly
    Hx = np.zeros((2, 2))
    for i in range(2):
        for j in range(2):
            bi, bj = prob.mps[i], prob.mps[j]
            hi = bi.U.T @ prob.h @ bi.U
            Li = np.einsum("pa,kpq,qb->kab", bi.U, prob.L, bi.U)
            Hf = fock.hamiltonian_fock(hi, np.einsum("kpq,krs->pqrs", Li, Li))
            vj = fock.rotation_matrix_fock(bi.U.T @ bj.U) @ fock.mps_to_vector(bj.sites)
            Hx[i, j] = fock.mps_to_vector(bi.sites) @ (Hf @ vj)
    assert np.abs(H - Hx).max() <= 1e-12 * np.abs(Hx).max()


def _with(prob, **kw):
    d = dict(prob.__dict__)
    d.update(kw)
    return synth.Problem(**d)


def test_edge_cases(ctx):
    base = synth.make_problem(5, 3, 1, 6, 3, 4, (31,))      # odd N, uneven spins
    # one MPS flipped to det U = -1 exercises the parity gate of the plan
    m2 = base.mps[2]
    U = m2.U.copy()
    U[:, 0] *= -1
    prob = _with(base, mps=[base.mps[0], base.mps[1], synth.MPS(m2.sites, m2.bond_qn, U)], e_core=1.25)
    for chi in (1, 2, 6):
        H, S, E, c, rep = ctx.subspace(prob, chi=chi)
        Ho, So, Eo, co, _ = oracle_subspace(prob, chi_cap=chi)
        _assert_pencil(H, S, E, Ho, So, Eo)
    # M = 1: Rayleigh quotient, no gates
    one = _with(base, mps=[base.mps[1]])
    H, S, E, c, rep = ctx.subspace(one, chi=4)
    assert abs(E - H[0, 0] / S[0, 0]) < 1e-12
    # duplicated MPS: S singular, the duplicate is dropped
    dup = _with(base, mps=[base.mps[0], base.mps[1], base.mps[1]])
    H3, S3, E3, _, r3 = ctx.subspace(dup, chi=6)
    H2, S2, E2, _, r2 = ctx.subspace(_with(base, mps=[base.mps[0], base.mps[1]]), chi=6)
    assert r3["n_dropped"] == 1 and r2["n_dropped"] == 0
    assert abs(E3 - E2) < 1e-9


def test_determinants_match_slater_condon_full_size(ctx):
    """chi = 1 determinants at N = 24 sharing one basis (U = I, so every gate
    angle is zero and nothing is truncated): the pencil equals the
    Slater-Condon closed forms, independently of the oracle's MPO -- the
    diagonal, single and double excitations of both spin patterns."""
    from test_oracle_mpo import _det_mps, _slater_condon
    N = 24
    base = synth.make_problem(N, N // 2, N // 2, 4, 1, 8, (9, N))
    r = np.random.default_rng(N)
    occ = set(r.choice(np.arange(0, 2 * N, 2), N // 2, replace=False)) | \
        set(r.choice(np.arange(1, 2 * N, 2), N // 2, replace=False))
    occ = {int(x) for x in occ}
    up_occ = sorted(m for m in occ if m % 2 == 0)
    up_vir = sorted(m for m in range(0, 2 * N, 2) if m not in occ)
    dn_occ = sorted(m for m in occ if m % 2 == 1)
    dn_vir = sorted(m for m in range(1, 2 * N, 2) if m not in occ)
    dets = [occ,
            (occ - {up_occ[0]}) | {up_vir[-1]},
            (occ - {dn_occ[-1]}) | {dn_vir[0]},
            (occ - {up_occ[1], dn_occ[0]}) | {up_vir[0], dn_vir[-1]},
            (occ - {up_occ[0], up_occ[-1]}) | {up_vir[0], up_vir[-1]}]
    mps = []
    for d in dets:
        sites, qn = _det_mps(N, d)
        mps.append(synth.MPS(sites=sites, bond_qn=qn, U=np.eye(N)))
    prob = _with(base, mps=mps, chi=1)
    H, S, E, c, rep = ctx.subspace(prob, chi=1)
    h, g = prob.h, prob.g()
    for i in range(len(dets)):
        for j in range(len(dets)):
            want = _slater_condon(h, g, sorted(dets[i]), sorted(dets[j]))
            assert abs(H[i, j] - want) <= 1e-11 * max(1.0, abs(want)), (i, j, H[i, j], want)
    np.testing.assert_allclose(S, np.eye(len(dets)), rtol=0, atol=1e-13)


def test_input_validation(ctx):
    base = synth.make_problem(4, 2, 2, 4, 2, 3, (32,))
    bad_u = _with(base, mps=[base.mps[0], synth.MPS(base.mps[1].sites, base.mps[1].bond_qn, base.mps[1].U * 1.01)])
    with pytest.raises(T.TnqeError) as e:
        ctx.subspace(bad_u, chi=4)
    assert e.value.status == -3
    sites = [a.copy() for a in base.mps[0].sites]
    sites[1][0, 0, :] = 1.0                                        # breaks the blocks
    with pytest.raises(T.TnqeError) as e:
        ctx.subspace(_with(base, mps=[synth.MPS(sites, base.mps[0].bond_qn, base.mps[0].U)]), chi=4)
    assert e.value.status == -4
    # the same checks on the second MPS of two (scanned by another host worker)
    sites = [a.copy() for a in base.mps[1].sites]
    sites[2][0, 0, :] = 1.0
    with pytest.raises(T.TnqeError) as e:
        ctx.subspace(_with(base, mps=[base.mps[0], synth.MPS(sites, base.mps[1].bond_qn, base.mps[1].U)]), chi=4)
    assert e.value.status == -4
    sites = [a.copy() for a in base.mps[1].sites]
    sites[-1].flat[0] = np.inf
    with pytest.raises(T.TnqeError) as e:
        ctx.subspace(_with(base, mps=[base.mps[0], synth.MPS(sites, base.mps[1].bond_qn, base.mps[1].U)]), chi=4)
    assert e.value.status == -9
    h = base.h.copy()
    h[0, 0] = np.nan
    with pytest.raises(T.TnqeError) as e:
        ctx.subspace(_with(base, h=h), chi=4)
    assert e.value.status in (-1, -9)
    # the context still works after errors
    H, S, E, c, rep = ctx.subspace(base, chi=4)
    assert np.isfinite(E)


def test_fp32_environments(ctx):
    """All environments in FP32 (every pair): each element against the FP64
    oracle relative to itself, and the eigenvalue error reported.  Plain FP32
    storage does not reach the 1e-6 Ha target at this size (the diagonal
    elements are ~60 Ha and FP32 keeps ~7 digits); see the xfail below."""
    prob = synth.make_config(3)
    g = np.load(os.path.join(GOLD, "oracle_config3.npz"))
    H, S, E, c, rep = ctx.subspace(prob, chi=prob.chi, precision="fp32")
    dE = abs(E - float(g["E"]))
    relH = np.max(np.abs(H - g["H"]) / np.abs(g["H"]))
    relS = np.max(np.abs(S - g["S"]) / np.abs(g["S"]))
    print(f"fp32: dE={dE:.2e} max_rel_dH={relH:.2e} max_rel_dS={relS:.2e}", flush=True)
    assert rep["n_fp32_pairs"] == prob.M * (prob.M + 1) // 2
    # FP32 rounding over 12 sites of environment contractions: 1e-4 relative
    # to each element (measured ~1e-6 on the diagonal)
    assert relH < 1e-4 and relS < 1e-4
    assert dE < 1e-4


@pytest.mark.xfail(strict=True, reason="plain FP32 environments miss |dE| <= 1e-6 Ha (measured ~3e-6 at N = 12)")
def test_fp32_environments_meet_target(ctx):
    prob = synth.make_config(3)
    g = np.load(os.path.join(GOLD, "oracle_config3.npz"))
    H, S, E, c, rep = ctx.subspace(prob, chi=prob.chi, precision="fp32")
    assert abs(E - float(g["E"])) <= 1e-6


def test_reduced_precision_modes(ctx):
    """Every pair in reduced precision at N = 12, chi = 64.  FP32 on the
    shifted operator H - c N meets |dE| <= 1e-6 Ha; the BF16 modes are
    measured against the FP64 oracle and bounded by their arithmetic (BF16
    keeps 8 bits, split BF16 about 16)."""
    prob = synth.make_config(3)
    g = np.load(os.path.join(GOLD, "oracle_config3.npz"))
    hmax = np.abs(g["H"]).max()
    for prec, e_tol, h_tol in (("fp32_shift", 1e-6, 1e-6), ("bf16x3", 1e-3, 1e-4), ("bf16", 1e-1, 2e-2)):
        H, S, E, c, rep = ctx.subspace(prob, chi=prob.chi, precision=prec)
        dE = abs(E - float(g["E"]))
        dH = np.abs(H - g["H"]).max() / hmax
        dS = np.abs(S - g["S"]).max()
        print(f"{prec}: dE={dE:.2e} dH_rel={dH:.2e} dS={dS:.2e}", flush=True)
        assert rep["n_fp32_pairs"] == prob.M * (prob.M + 1) // 2
        assert dE <= e_tol and dH <= h_tol
        np.testing.assert_array_equal(H, H.T)


@pytest.mark.xfail(strict=True, reason="FP32 on the shifted operator misses |dE| <= 1e-6 Ha at N = 24 (measured 1.4e-6)")
def test_fp32_shift_full_size_target(ctx):
    prob = synth.make_config(5)
    up = ctx.upload(prob)
    try:
        H, S, E, c, rep = up.solve(chi=prob.chi)
        Hm, Sm, Em, cm, repm = up.solve(chi=prob.chi, precision="fp32_shift")
    finally:
        up.free()
    assert abs(Em - E) <= 1e-6


def test_full_size_sampled_pairs(ctx):
    """N = 24, chi = 256, M = 16: the benchmark workload, checked on sampled pairs."""
    prob = synth.make_config(5)
    g = np.load(os.path.join(GOLD, "oracle_config5_pairs.npz"))
    H, S, E, c, rep = ctx.subspace(prob, chi=prob.chi)
    for key in g.files:
        i, j = map(int, key.split("_"))
        h, s = g[key][0], g[key][1]
        print(f"pair {i},{j}: dH={abs(H[i, j] - h):.2e} dS={abs(S[i, j] - s):.2e}")
        # each sampled element relative to itself (off-diagonal elements are
        # ~1e-8 of the diagonal ones at this size)
        assert abs(H[i, j] - h) <= RTOL * abs(h)
        assert abs(S[i, j] - s) <= RTOL * abs(s)
    np.testing.assert_allclose(np.diag(S), 1.0, atol=1e-12)
    assert rep["max_discarded_weight_sum"] <= 1.0 + 1e-9


def test_dense_coupling_path(monkeypatch):
    """Every MPO coupling routed through the dense mixing GEMMs (N = 7)."""
    monkeypatch.setenv("TNQE_DENSE_MIN_AREA", "1")
    c = T.Context(0)
    try:
        prob = synth.make_config(2)
        g = np.load(os.path.join(GOLD, "oracle_config2.npz"))
        for prec, tol in (("fp64", RTOL), ("fp32", 1e-5)):
            H, S, E, cv, rep = c.subspace(prob, chi=prob.chi, precision=prec)
            _assert_pencil(H, S, E, g["H"], g["S"], float(g["E"]), tol)
    finally:
        c.close()


def test_batch_of_subspaces(ctx):
    """64 independent subspaces (N in 8..16, chi in {16..128}, M in 2..8) in
    one batched call; sampled subspaces (every chi, H by sector FCI up to
    N = 13) against the stored oracle values, element by element."""
    probs = synth.make_batch()
    g = np.load(os.path.join(GOLD, "oracle_batch.npz"))
    ups = [ctx.upload(p) for p in probs]
    try:
        Hs, Ss, Es, reps = ctx.solve_batch(ups, [p.chi for p in probs])
    finally:
        for u in ups:
            u.free()
    assert len(Hs) == len(probs)
    for s_ in range(len(probs)):
        assert np.isfinite(Es[s_])
        np.testing.assert_allclose(np.diag(Ss[s_]), 1.0, atol=1e-12)
    sampled = sorted({int(k[1:]) for k in g.files if k.startswith("E")})
    assert {probs[s_].chi for s_ in sampled} == {16, 32, 64, 128} and len(sampled) >= 8
    for s_ in sampled:
        print(f"subspace {s_}: N={probs[s_].N} chi={probs[s_].chi} M={probs[s_].M} ({g[f'method{s_}']})",
              flush=True)
        _assert_pencil(Hs[s_], Ss[s_], Es[s_], g[f"H{s_}"], g[f"S{s_}"], float(g[f"E{s_}"]), elementwise=True)
        _assert_report(reps[s_], g[f"H{s_}"], g[f"S{s_}"])
        assert abs(reps[s_]["max_discarded_weight_sum"] - float(g[f"rep{s_}"][5])) < 1e-10


def test_subspace_batch_with_workspace(ctx):
    """tnqe_subspace_batch from host inputs, all subspaces in one caller
    workspace (the largest bound of the set)."""
    import torch
    probs = synth.make_batch()
    g = np.load(os.path.join(GOLD, "oracle_batch.npz"))
    sampled = sorted({int(k[1:]) for k in g.files if k.startswith("E")})
    sel = [probs[s_] for s_ in sampled]
    n = max(ctx.workspace_size(p, chi=p.chi) for p in sel)
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    Hs, Ss, Es, reps = ctx.subspace_batch(sel, workspace=ws)
    for s_, H, S, E, r in zip(sampled, Hs, Ss, Es, reps):
        _assert_pencil(H, S, E, g[f"H{s_}"], g[f"S{s_}"], float(g[f"E{s_}"]), elementwise=True)
        assert 0 < r["ws_peak_bytes"] <= n


def test_mixed_precision_full_size(ctx):
    """Mixed mode at N = 24: FP32 environments for the pairs whose rotated ket
    keeps <= 1e-6 of its squared norm; E within 1e-6 Ha of the FP64 path."""
    prob = synth.make_config(5)
    up = ctx.upload(prob)
    try:
        H, S, E, c, rep = up.solve(chi=prob.chi)
        Hm, Sm, Em, cm, repm = up.solve(chi=prob.chi, precision="mixed")
    finally:
        up.free()
    print(f"mixed: {repm['n_fp32_pairs']} FP32 pairs, dE={abs(Em - E):.2e}", flush=True)
    assert repm["n_fp32_pairs"] > 0
    assert abs(Em - E) <= 1e-6
    # FP64 pairs (the diagonal) agree to the FP64 tolerance
    np.testing.assert_allclose(np.diag(Hm), np.diag(H), rtol=1e-12)
    np.testing.assert_allclose(np.diag(Sm), np.diag(S), rtol=1e-12)
    # every FP32 element relative to itself, with no absolute floor: FP32
    # environments over 24 sites keep ~5 digits (measured <= 7e-5)
    off = ~np.eye(prob.M, dtype=bool)
    relH = np.abs(Hm - H)[off] / np.abs(H)[off]
    relS = np.abs(Sm - S)[off] / np.abs(S)[off]
    print(f"mixed FP32 elements: max_rel_dH={relH.max():.2e} max_rel_dS={relS.max():.2e}", flush=True)
    assert relH.max() < 1e-3 and relS.max() < 1e-3


def test_autotuned_tiles(ctx, tmp_path, monkeypatch):
    """Tile shapes of the environment GEMMs picked by timing (autotune = 1),
    cached on disk: the same pencil bit for bit (the K order of every output
    does not depend on the tile), and a second call tunes nothing."""
    monkeypatch.setenv("TNQE_TUNE_FILE", str(tmp_path / "tiles.txt"))
    c = T.Context(0)
    try:
        prob = synth.make_config(3)
        H0, S0, E0, _, _ = c.subspace(prob, chi=prob.chi)
        H1, S1, E1, _, r1 = c.subspace(prob, chi=prob.chi, autotune=True)
        lines = (tmp_path / "tiles.txt").read_text().split("\n")
        assert r1["t_tune_ms"] > 0 and len([x for x in lines if x.strip()]) > 0
        np.testing.assert_array_equal(H1, H0)
        np.testing.assert_array_equal(S1, S0)
        H2, S2, E2, _, r2 = c.subspace(prob, chi=prob.chi, autotune=True)
        assert r2["t_tune_ms"] < 0.2 * r1["t_tune_ms"]
        np.testing.assert_array_equal(H2, H0)
        c2 = T.Context(0)          # a new context reads the cached table
        try:
            H3, _, _, _, r3 = c2.subspace(prob, chi=prob.chi, autotune=True)
            assert r3["t_tune_ms"] < 0.2 * r1["t_tune_ms"]
            np.testing.assert_array_equal(H3, H0)
        finally:
            c2.close()
    finally:
        c.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3"])
def test_every_tile_shape(ctx, precision):
    """Every tile shape of the environment GEMMs forced on all of them
    (tile mode 2 + k): the pencil bit for bit the same as with the shape
    rule, in FP64 and in the FP32 and split-BF16 matrix-core variants."""
    prob = synth.make_config(3)
    H0, S0, _, _, _ = ctx.subspace(prob, chi=prob.chi, precision=precision)
    for k in range(5):
        print(f"tile candidate {k}, {precision}", flush=True)
        H, S, _, _, _ = ctx.subspace(prob, chi=prob.chi, precision=precision, autotune=2 + k)
        np.testing.assert_array_equal(H, H0)
        np.testing.assert_array_equal(S, S0)
    with pytest.raises(T.TnqeError):
        ctx.subspace(prob, chi=prob.chi, autotune=7)


def test_batch_concurrent_equals_sequential(ctx):
    """Concurrent subspaces (worker contexts on their own streams) give the
    same pencils as one after another."""
    probs = synth.make_batch()[:12]
    ups = [ctx.upload(p) for p in probs]
    try:
        Hs1, Ss1, Es1, _ = ctx.solve_batch(ups, [p.chi for p in probs], workers=1)
        Hs4, Ss4, Es4, _ = ctx.solve_batch(ups, [p.chi for p in probs], workers=4)
    finally:
        for u in ups:
            u.free()
    for a, b in zip(Hs1, Hs4):
        np.testing.assert_array_equal(a, b)
    for a, b in zip(Ss1, Ss4):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(Es1, Es4)
