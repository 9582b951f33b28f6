"""C-ABI library on the CPU: it loads, exports what include/tnqe.h declares, and
its host logic (Givens plan, d=4 gate, MPO) matches the oracle.  No device."""
import os
import re

import numpy as np
import pytest

import paper_2404_10223_amd as T
import tnqe_synth as synth
from oracle import fock, gates, givens

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "tnqe.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tnqe_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(T.LIB_PATH):
        from paper_2404_10223_amd.build import build
        build()
    return T.lib()


def test_exports_every_declared_symbol(lib):
    names = _declared_symbols()
    assert "tnqe_solve" in names and "tnqe_upload" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(T.EXPORTS) <= set(names)


def test_status_strings_and_options(lib):
    assert lib.tnqe_status_string(0) == b"ok"
    assert lib.tnqe_status_string(-3) == b"rotation is not orthogonal"
    o = T.options(chi=7)
    assert o.chi == 7 and o.eps_S == 1e-12 and o.tau_w == 1e-13


def test_create_without_device_fails_cleanly(lib):
    import ctypes as C
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    h = C.c_void_p()
    assert lib.tnqe_create(C.byref(h), 0, None) == -10   # TNQE_ENODEVICE


@pytest.mark.parametrize("N,det", [(2, 1), (4, 1), (7, -1), (24, 1)])
def test_host_givens_plan_matches_oracle(lib, N, det):
    r = np.random.default_rng(N)
    Q, R = np.linalg.qr(r.normal(size=(N, N)))
    Q = Q * np.sign(np.diag(R))
    if np.linalg.det(Q) * det < 0:
        Q[:, 0] *= -1
    gl, d = T.debug_givens(Q)
    go, do = givens.plan(Q)
    assert d == do
    assert [a for a, _ in gl] == [a for a, _ in go]
    np.testing.assert_allclose([t for _, t in gl], [t for _, t in go], atol=1e-13)
    np.testing.assert_allclose(givens.compose(N, gl, d), Q, atol=1e-12)


def test_host_gate_matches_oracle(lib):
    for th in (0.0, 0.31, -2.2, np.pi / 2):
        np.testing.assert_allclose(T.debug_gate(th), gates.g4(th), atol=1e-15)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_host_mpo_contracts_to_fock_hamiltonian(lib, N):
    prob = synth.make_problem(N, min(1, N), min(1, N), 2, 1, 3, (77, N))
    g = prob.g()
    H, I, mb = T.debug_mpo_dense(prob.h, g)
    np.testing.assert_allclose(H, fock.hamiltonian_fock(prob.h, g).toarray(), atol=1e-12)
    np.testing.assert_array_equal(I, np.eye(4 ** N))
    assert mb <= 2 + 4 * N + 8 * (N // 2) ** 2 + 2 * N


@pytest.mark.parametrize("N", [3, 5])
def test_host_mpo_dense_coupling_blocks(lib, N, monkeypatch):
    # every coupling stored as a dense block: the same Hamiltonian
    monkeypatch.setenv("TNQE_DENSE_MIN_AREA", "1")
    prob = synth.make_problem(N, 1, 1, 2, 1, 3, (78, N))
    g = prob.g()
    H, I, _ = T.debug_mpo_dense(prob.h, g)
    np.testing.assert_allclose(H, fock.hamiltonian_fock(prob.h, g).toarray(), atol=1e-12)


def test_host_pool_back_to_back_jobs():
    """The host worker pool under many short back-to-back loops: a worker that
    wakes after its loop has returned must not run the next loop's items with
    the old function (every item runs exactly once)."""
    jobs = 20000
    assert T.debug_host_pool(7, jobs) == sum(1 + j % 5 for j in range(jobs))
    assert T.debug_host_pool(0, 100) == sum(1 + j % 5 for j in range(100))



def test_workspace_size_host_only(lib):
    """tnqe_workspace_size needs no device: it validates the inputs and bounds
    the device memory of a call; the bound covers at least the inputs and the
    rotated kets, grows with chi, and rejects bad inputs like a solve."""
    p1, p2 = synth.make_config(1), synth.make_config(2)
    b1 = T.workspace_size(p1, chi=p1.chi)
    sites = sum(a.size for m in p1.mps for a in m.sites) * 8
    assert b1 > sites
    small, large = T.workspace_size(p2, chi=4), T.workspace_size(p2, chi=16)
    assert 0 < small < large
    # FP32 environments need no more than FP64 ones
    assert T.workspace_size(p2, chi=16, precision="fp32") <= large
    # the full-size workload: bounded well inside one GPU's 288 GB
    p5 = synth.make_config(5)
    assert T.workspace_size(p5, chi=p5.chi) < 64 * 2 ** 30
    bad = synth.Problem(**{**p1.__dict__, "mps": [synth.MPS(p1.mps[0].sites, p1.mps[0].bond_qn,
                                                             p1.mps[0].U * 1.01)]})
    with pytest.raises(T.TnqeError) as e:
        T.workspace_size(bad, chi=4)
    assert e.value.status == -3
    with pytest.raises(T.TnqeError):
        T.workspace_size(p1, chi=0)


def test_onehot_size_matches_oracle(lib):
    """Number of one-hot states of the expanded pencil (host-only) against the
    oracle's enumeration of the particle-number-conserving entries."""
    from oracle.onehot import onehot_pencil
    for k, i, p in [(1, 1, 1), (2, 2, 3), (2, 0, 0), (2, 3, 5)]:
        prob = synth.make_config(k)
        assert T.onehot_size(prob, i, p, chi=prob.chi) == len(onehot_pencil(prob, i, p)[0])
    prob = synth.make_config(1)
    with pytest.raises(T.TnqeError):
        T.onehot_size(prob, 2, 0, chi=4)
    with pytest.raises(T.TnqeError):
        T.onehot_size(prob, 0, 3, chi=4)
