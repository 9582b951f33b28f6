"""Python binding of libtnqe.so (ctypes; argument marshalling only).

Every step of the computation runs in the HIP library; this module only packs
NumPy arrays into the C structs declared in include/tnqe.h, passes torch's
current HIP stream, and unpacks results.  It fails loudly when the library is
not built or no gfx950 device is present: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtnqe.so")

TNQE_FP64 = 0
TNQE_ENV_FP32 = 1
TNQE_ENV_MIXED = 2
TNQE_ENV_FP32_SHIFT = 3
TNQE_ENV_BF16 = 4
TNQE_ENV_BF16X3 = 5
PRECISIONS = {"fp64": TNQE_FP64, "fp32": TNQE_ENV_FP32, "mixed": TNQE_ENV_MIXED, "fp32_shift": TNQE_ENV_FP32_SHIFT,
              "bf16": TNQE_ENV_BF16, "bf16x3": TNQE_ENV_BF16X3}


class _Ham(C.Structure):
    _fields_ = [("N", C.c_int32), ("n_alpha", C.c_int32), ("n_beta", C.c_int32),
                ("h", C.POINTER(C.c_double)), ("n_chol", C.c_int32),
                ("L", C.POINTER(C.c_double)), ("g", C.POINTER(C.c_double)), ("e_core", C.c_double)]


class _Mps(C.Structure):
    _fields_ = [("bond_dim", C.POINTER(C.c_int32)), ("bond_qn", C.POINTER(C.c_int32)),
                ("sites", C.POINTER(C.c_double)), ("U", C.POINTER(C.c_double))]


class _Opts(C.Structure):
    _fields_ = [("chi", C.c_int32), ("chi_cap_override", C.c_int32), ("precision", C.c_int32),
                ("eps_S", C.c_double), ("tau_w", C.c_double), ("max_sweeps", C.c_int32),
                ("renormalize", C.c_int32), ("autotune", C.c_int32), ("workers", C.c_int32),
                ("reserved", C.c_int32 * 4)]


class _SweepOpts(C.Structure):
    _fields_ = [("rotation", C.c_int32), ("n_grid", C.c_int32), ("n_golden", C.c_int32), ("nreps", C.c_int32),
                ("tol_ld", C.c_double), ("e_tol", C.c_double), ("reserved", C.c_double * 2)]


class _SweepRes(C.Structure):
    _fields_ = [("E_old", C.c_double), ("E1", C.c_double), ("theta", C.c_double), ("xi_none", C.c_double),
                ("xi", C.c_double), ("discarded", C.c_double), ("n_onehot", C.c_int32),
                ("n_columns", C.c_int32), ("n_kept", C.c_int32), ("n_dropped_S", C.c_int32),
                ("accepted", C.c_int32), ("new_bond", C.c_int32), ("mit_columns", C.c_int32),
                ("mit_kept", C.c_int32), ("E_new", C.c_double)]


ROTATIONS = {"none": 0, "fswap": 1, "givens": 2}


class _Report(C.Structure):
    _fields_ = [("max_discarded_weight_sum", C.c_double), ("min_rel_gap", C.c_double),
                ("cond_S", C.c_double), ("lambda_min_S", C.c_double), ("kappa1", C.c_double),
                ("t_total_ms", C.c_double), ("t_host_ms", C.c_double), ("t_gates_ms", C.c_double),
                ("t_env_ms", C.c_double), ("t_gep_ms", C.c_double), ("alg_flops", C.c_double),
                ("alg_bytes", C.c_double), ("env_flops", C.c_double), ("env_kernel_ms", C.c_double),
                ("svd_kernel_ms", C.c_double), ("svd_flops", C.c_double),
                ("svd_kind_ms", C.c_double * 16), ("svd_kind_flops", C.c_double * 16),
                ("env_kind_ms", C.c_double * 8), ("env_kind_flops", C.c_double * 8),
                ("env_kind_bytes", C.c_double * 8),
                ("n_dropped", C.c_int32), ("n_pairs", C.c_int32), ("max_bond", C.c_int32),
                ("mpo_max_bond", C.c_int32), ("svd_launches", C.c_int32),
                ("svd_kind_launches", C.c_int32 * 16), ("env_kind_launches", C.c_int32 * 8),
                ("n_fp32_pairs", C.c_int32),
                ("reserved", C.c_int32 * 7), ("ws_peak_bytes", C.c_double),
                ("move_kernel_ms", C.c_double), ("move_flops", C.c_double), ("t_moves_ms", C.c_double),
                ("t_tune_ms", C.c_double), ("move_launches", C.c_int32), ("reserved2", C.c_int32)]


EXPORTS = ["tnqe_default_options", "tnqe_create", "tnqe_destroy", "tnqe_trim", "tnqe_upload",
           "tnqe_problem_free", "tnqe_solve", "tnqe_solve_batch", "tnqe_workspace_size", "tnqe_subspace",
           "tnqe_subspace_batch", "tnqe_status_string", "tnqe_last_error", "tnqe_version", "tnqe_debug_givens",
           "tnqe_debug_gate", "tnqe_debug_mpo_dense", "tnqe_debug_host_pool", "tnqe_debug_select",
           "tnqe_debug_gep", "tnqe_subspace_noalloc", "tnqe_noalloc_capacity", "tnqe_onehot_size",
           "tnqe_onehot_pencil", "tnqe_sweep_step", "tnqe_sweep_last_params", "tnqe_debug_psd_eigen"]

_lib = None


def lib():
    """Load libtnqe.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2404_10223_amd/build.py")
    # torch ships its own HIP runtime under the same soname; loading it first
    # makes the library bind to that one runtime, so torch's streams and ours
    # are the same objects
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, ip = C.c_void_p, C.c_int32
    dp = C.POINTER(C.c_double)
    L.tnqe_default_options.argtypes = [C.POINTER(_Opts)]
    L.tnqe_default_options.restype = None
    L.tnqe_create.argtypes = [C.POINTER(vp), C.c_int, vp]
    L.tnqe_destroy.argtypes = [vp]
    L.tnqe_trim.argtypes = [vp]
    L.tnqe_upload.argtypes = [vp, C.POINTER(_Ham), ip, C.POINTER(_Mps), C.POINTER(vp)]
    L.tnqe_problem_free.argtypes = [vp]
    L.tnqe_solve.argtypes = [vp, vp, C.POINTER(_Opts), dp, dp, dp, dp, C.POINTER(_Report)]
    L.tnqe_solve_batch.argtypes = [vp, ip, C.POINTER(vp), C.POINTER(_Opts), C.POINTER(dp), C.POINTER(dp),
                                   dp, C.POINTER(_Report)]
    L.tnqe_workspace_size.argtypes = [vp, C.POINTER(_Ham), ip, C.POINTER(_Mps), C.POINTER(_Opts),
                                      C.POINTER(C.c_size_t)]
    L.tnqe_subspace.argtypes = [vp, C.POINTER(_Ham), ip, C.POINTER(_Mps), C.POINTER(_Opts), vp, C.c_size_t,
                                dp, dp, dp, dp, C.POINTER(_Report)]
    L.tnqe_subspace_batch.argtypes = [vp, ip, C.POINTER(_Ham), C.POINTER(ip), C.POINTER(C.POINTER(_Mps)),
                                      C.POINTER(_Opts), vp, C.c_size_t, C.POINTER(dp), C.POINTER(dp), dp,
                                      C.POINTER(_Report)]
    L.tnqe_debug_gep.argtypes = [vp, ip, dp, dp, C.c_double, dp]
    L.tnqe_subspace_noalloc.argtypes = [vp, C.POINTER(_Ham), ip, C.POINTER(_Mps), C.POINTER(_Opts), dp, dp, dp, dp,
                                        C.POINTER(_Report)]
    L.tnqe_onehot_size.argtypes = [vp, C.POINTER(_Ham), ip, C.POINTER(_Mps), C.POINTER(_Opts), ip, ip,
                                   C.POINTER(ip)]
    L.tnqe_onehot_pencil.argtypes = [vp, C.POINTER(_Ham), ip, C.POINTER(_Mps), C.POINTER(_Opts), ip, ip, ip,
                                     C.POINTER(ip), dp, dp, dp, dp, C.POINTER(_Report)]
    L.tnqe_sweep_step.argtypes = [vp, C.POINTER(_Ham), ip, C.POINTER(_Mps), C.POINTER(_Opts), C.POINTER(_SweepOpts),
                                  ip, ip, dp, dp, C.POINTER(ip), C.POINTER(ip), C.c_int64, dp, C.c_int64, dp,
                                  C.POINTER(_SweepRes), C.POINTER(_Report)]
    L.tnqe_sweep_last_params.argtypes = [vp, ip, dp]
    L.tnqe_debug_psd_eigen.argtypes = [vp, ip, dp, ip, ip, dp, dp]
    L.tnqe_noalloc_capacity.argtypes = []
    L.tnqe_noalloc_capacity.restype = C.c_size_t
    L.tnqe_status_string.argtypes = [C.c_int]
    L.tnqe_status_string.restype = C.c_char_p
    L.tnqe_last_error.argtypes = [vp]
    L.tnqe_last_error.restype = C.c_char_p
    L.tnqe_version.restype = C.c_char_p
    L.tnqe_debug_givens.argtypes = [ip, dp, C.POINTER(C.c_int32), dp, C.POINTER(C.c_int32)]
    L.tnqe_debug_gate.argtypes = [C.c_double, dp]
    L.tnqe_debug_mpo_dense.argtypes = [ip, dp, dp, dp, dp, C.POINTER(C.c_int32)]
    L.tnqe_debug_host_pool.argtypes = [ip, ip, C.POINTER(C.c_int64)]
    L.tnqe_debug_select.argtypes = [vp, ip, C.POINTER(C.c_int32), C.POINTER(C.c_int32), dp, ip, C.c_double,
                                    C.POINTER(C.c_int32), dp]
    for name in EXPORTS:
        getattr(L, name)
    _lib = L
    return L


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


class TnqeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"tnqe status {status}: {msg}")
        self.status = status


def _check(st, ctx=None):
    if st != 0:
        L = lib()
        msg = L.tnqe_last_error(ctx).decode() if ctx else ""
        raise TnqeError(st, f"{L.tnqe_status_string(st).decode()}: {msg}")


def options(chi=16, precision="fp64", chi_cap_override=0, eps_S=1e-12, tau_w=1e-13, max_sweeps=40,
            renormalize=False, autotune=False, workers=0):
    o = _Opts()
    lib().tnqe_default_options(C.byref(o))
    o.chi = chi
    o.chi_cap_override = chi_cap_override
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.eps_S = eps_S
    o.tau_w = tau_w
    o.max_sweeps = max_sweeps
    o.renormalize = int(bool(renormalize))
    o.autotune = int(autotune)   # False/0 rule, True/1 tuned, 2 + k tile candidate k
    o.workers = int(workers)
    return o


def _ptr(buf):
    """(device address, bytes) of a workspace given as a torch tensor, or (None, 0)."""
    if buf is None:
        return None, 0
    if isinstance(buf, int):
        raise TypeError("pass the workspace as a torch tensor")
    return C.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size()


def workspace_size(prob, ctx=None, **kw):
    """Device bytes that always suffice for a workspace call (host-side only:
    works without a GPU when ctx is None)."""
    pk = _Packed(prob)
    o = options(**kw)
    out = C.c_size_t(0)
    h = ctx.h if ctx is not None else None
    _check(lib().tnqe_workspace_size(h, C.byref(pk.ham), prob.M, pk.mps, C.byref(o), C.byref(out)), h)
    return out.value


def onehot_size(prob, i, p, **kw):
    """Number of one-hot states of state i at sites (p, p+1) (host-only)."""
    pk = _Packed(prob)
    o = options(**kw)
    n = C.c_int32(0)
    _check(lib().tnqe_onehot_size(None, C.byref(pk.ham), prob.M, pk.mps, C.byref(o), int(i), int(p), C.byref(n)))
    return n.value


def report_dict(r):
    out = {}
    for name, _ in _Report._fields_:
        if name.startswith("reserved"):
            continue
        v = getattr(r, name)
        out[name] = list(v) if isinstance(v, C.Array) else v
    return out


class _Packed:
    """Keeps the NumPy buffers alive while the C structs point at them."""

    def __init__(self, prob):
        self.h = np.ascontiguousarray(prob.h, dtype=np.float64)
        self.L = np.ascontiguousarray(prob.L, dtype=np.float64)
        self.ham = _Ham(prob.N, prob.n_alpha, prob.n_beta, _dptr(self.h), self.L.shape[0], _dptr(self.L),
                        None, float(prob.e_core))
        self.keep = []
        arr = (_Mps * prob.M)()
        for i, m in enumerate(prob.mps):
            dims = np.array([q.shape[0] for q in m.bond_qn], dtype=np.int32)
            qn = np.ascontiguousarray(np.concatenate([np.asarray(q, dtype=np.int32).reshape(-1, 2)
                                                      for q in m.bond_qn]))
            sites = np.ascontiguousarray(np.concatenate([np.asarray(a, dtype=np.float64).reshape(-1)
                                                         for a in m.sites]))
            U = np.ascontiguousarray(m.U, dtype=np.float64)
            self.keep += [dims, qn, sites, U]
            arr[i] = _Mps(_iptr(dims), _iptr(qn), _dptr(sites), _dptr(U))
        self.mps = arr


class Context:
    """A library context on one GPU, issuing work on torch's current stream."""

    def __init__(self, device=0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible to torch")
        torch.cuda.set_device(device)
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        self.L = lib()
        h = C.c_void_p()
        _check(self.L.tnqe_create(C.byref(h), device, C.c_void_p(stream)))
        self.h = h

    def close(self):
        if self.h:
            self.L.tnqe_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def upload(self, prob):
        pk = _Packed(prob)
        out = C.c_void_p()
        _check(self.L.tnqe_upload(self.h, C.byref(pk.ham), prob.M, pk.mps, C.byref(out)), self.h)
        return Uploaded(self, out, prob.M)

    def subspace(self, prob, workspace=None, **kw):
        """One call from host inputs (tnqe_subspace).  workspace: a torch
        device tensor the call takes all its device memory from, or None (the
        context's pool)."""
        pk = _Packed(prob)
        o = options(**kw)
        M = prob.M
        H = np.zeros((M, M))
        S = np.zeros((M, M))
        E = np.zeros(1)
        c = np.zeros(M)
        r = _Report()
        wp, wb = _ptr(workspace)
        _check(self.L.tnqe_subspace(self.h, C.byref(pk.ham), M, pk.mps, C.byref(o), wp, wb, _dptr(H), _dptr(S),
                                    _dptr(E), _dptr(c), C.byref(r)), self.h)
        return H, S, float(E[0]), c, report_dict(r)

    def workspace_size(self, prob, **kw):
        return workspace_size(prob, self, **kw)

    def onehot_pencil(self, prob, i, p, **kw):
        """Expanded one-hot pencil of state i at sites (p, p+1): (index [n][4],
        Hd, Sd [n][n], Hc, Sc [n][M], report)."""
        pk = _Packed(prob)
        o = options(**kw)
        n = C.c_int32(0)
        _check(self.L.tnqe_onehot_size(self.h, C.byref(pk.ham), prob.M, pk.mps, C.byref(o), int(i), int(p),
                                       C.byref(n)), self.h)
        n = n.value
        index = np.zeros((n, 4), dtype=np.int32)
        Hd, Sd = np.zeros((n, n)), np.zeros((n, n))
        Hc, Sc = np.zeros((n, prob.M)), np.zeros((n, prob.M))
        r = _Report()
        _check(self.L.tnqe_onehot_pencil(self.h, C.byref(pk.ham), prob.M, pk.mps, C.byref(o), int(i), int(p), n,
                                         _iptr(index), _dptr(Hd), _dptr(Sd), _dptr(Hc), _dptr(Sc), C.byref(r)),
               self.h)
        return index, Hd, Sd, Hc, Sc, report_dict(r)

    def sweep_step(self, prob, H, S, i, p, rotation="none", tol_ld=1e-3, e_tol=0.0, n_grid=36, n_golden=40, nreps=0,
                   **kw):
        """One generalized-sweep step at sites (p, p+1) for state i
        (tnqe_sweep_step).  H, S: the current pencil.  Returns (result dict,
        the updated state as an MPS-like (sites, bond_qn, U) triple, t' [n],
        report)."""
        pk = _Packed(prob)
        o = options(**kw)
        so = _SweepOpts(ROTATIONS[rotation], int(n_grid), int(n_golden), int(nreps), float(tol_ld), float(e_tol))
        m = prob.mps[i]
        N = prob.N
        chi = o.chi_cap_override if o.chi_cap_override > 0 else o.chi
        dims_in = [q.shape[0] for q in m.bond_qn]
        qn_cap = sum(dims_in) + chi
        # (an out-of-range p is the library's to reject)
        edge = dims_in[min(max(p, 0), N)] + dims_in[min(max(p + 2, 0), N)]
        sites_cap = sum(a.size for a in m.sites) + 4 * chi * edge
        bond_dim = np.zeros(N + 1, dtype=np.int32)
        bond_qn = np.zeros((qn_cap, 2), dtype=np.int32)
        sites = np.zeros(sites_cap)
        U = np.zeros((N, N))
        Hh = np.ascontiguousarray(H, dtype=np.float64)
        Sh = np.ascontiguousarray(S, dtype=np.float64)
        res = _SweepRes()
        r = _Report()
        _check(self.L.tnqe_sweep_step(self.h, C.byref(pk.ham), prob.M, pk.mps, C.byref(o), C.byref(so), int(i),
                                      int(p), _dptr(Hh), _dptr(Sh), _iptr(bond_dim), _iptr(bond_qn),
                                      int(qn_cap), _dptr(sites), int(sites_cap), _dptr(U), C.byref(res),
                                      C.byref(r)), self.h)
        out = {name: getattr(res, name) for name, _ in _SweepRes._fields_ if not name.startswith("reserved")}
        t = np.zeros(res.n_onehot)
        _check(self.L.tnqe_sweep_last_params(self.h, res.n_onehot, _dptr(t)), self.h)
        # unpack the state (layout of tnqe_mps)
        qns, st, o_q, o_s = [], [], 0, 0
        for b in range(N + 1):
            qns.append(bond_qn[o_q:o_q + bond_dim[b]].astype(np.int64).copy())
            o_q += bond_dim[b]
        for x in range(N):
            n = bond_dim[x] * 4 * bond_dim[x + 1]
            st.append(sites[o_s:o_s + n].reshape(bond_dim[x], 4, bond_dim[x + 1]).copy())
            o_s += n
        return out, (st, qns, U), t, report_dict(r)

    def subspace_noalloc(self, prob, **kw):
        """tnqe_subspace_noalloc: the library's fixed per-GPU scratch, no allocation."""
        pk = _Packed(prob)
        o = options(**kw)
        M = prob.M
        H = np.zeros((M, M))
        S = np.zeros((M, M))
        E = np.zeros(1)
        c = np.zeros(M)
        r = _Report()
        _check(self.L.tnqe_subspace_noalloc(self.h, C.byref(pk.ham), M, pk.mps, C.byref(o), _dptr(H), _dptr(S),
                                            _dptr(E), _dptr(c), C.byref(r)), self.h)
        return H, S, float(E[0]), c, report_dict(r)

    def subspace_batch(self, probs, chis=None, workspace=None, **kw):
        """Several subspaces from host inputs (tnqe_subspace_batch)."""
        n = len(probs)
        chis = [p.chi for p in probs] if chis is None else chis
        packs = [_Packed(p) for p in probs]
        hams = (_Ham * n)(*[pk.ham for pk in packs])
        Ms = np.array([p.M for p in probs], dtype=np.int32)
        mps = (C.POINTER(_Mps) * n)(*[C.cast(pk.mps, C.POINTER(_Mps)) for pk in packs])
        o = (_Opts * n)(*[options(chi=int(ch), **kw) for ch in chis])
        Hs = [np.zeros((p.M, p.M)) for p in probs]
        Ss = [np.zeros((p.M, p.M)) for p in probs]
        E = np.zeros(n)
        reps = (_Report * n)()
        hp = (C.POINTER(C.c_double) * n)(*[_dptr(x) for x in Hs])
        sp = (C.POINTER(C.c_double) * n)(*[_dptr(x) for x in Ss])
        wp, wb = _ptr(workspace)
        _check(self.L.tnqe_subspace_batch(self.h, n, hams, _iptr(Ms), mps, o, wp, wb, hp, sp, _dptr(E), reps),
               self.h)
        return Hs, Ss, E, [report_dict(r) for r in reps]

    def debug_gep(self, H, S, eps_S=1e-12):
        """Device eigensolver on a given pencil: dict of E, cond_S, lambda_min,
        n_dropped, kappa1, status and c."""
        H = np.ascontiguousarray(H, dtype=np.float64)
        S = np.ascontiguousarray(S, dtype=np.float64)
        M = H.shape[0]
        out = np.zeros(8 + M)
        _check(self.L.tnqe_debug_gep(self.h, M, _dptr(H), _dptr(S), float(eps_S), _dptr(out)), self.h)
        return dict(E=out[0], cond_S=out[1], lambda_min=out[2], n_dropped=int(out[3]), kappa1=out[4],
                    status=int(out[5]), c=out[8:8 + M].copy())

    def debug_psd_eigen(self, A, path=0, max_sweeps=40):
        """Device eigensolver of the sweep step's dense eigenproblems on a
        symmetric positive semi-definite A: (values in decreasing order,
        vectors by row).  path 0: the sweep step's choice, 1: one-workgroup
        global-memory Jacobi, 2: the same sweeps spread over the chip by
        column pairs, 3: spread over the chip by blocks of columns with each
        sweep replayed from a captured HIP graph, 4: as 3 with the launches
        issued one by one."""
        A = np.ascontiguousarray(A, dtype=np.float64)
        n = A.shape[0]
        vec, val = np.zeros((n, n)), np.zeros(n)
        _check(self.L.tnqe_debug_psd_eigen(self.h, n, _dptr(A), int(path), int(max_sweeps), _dptr(vec),
                                           _dptr(val)), self.h)
        return val, vec

    def debug_select(self, blocks, chi, tau):
        """Device truncation rule on given singular values: blocks[t] is the
        list of ket t's blocks, each a 1-D array sorted in decreasing order.
        Returns (kept counts per block, per ket: [keep, discarded, gap])."""
        nblk = np.array([len(b) for b in blocks], dtype=np.int32)
        n = np.array([len(x) for b in blocks for x in b], dtype=np.int32)
        flat = [np.asarray(x, dtype=np.float64) for b in blocks for x in b]
        sv = np.ascontiguousarray(np.concatenate(flat) if flat else np.zeros(1))
        kept = np.zeros(max(1, len(n)), dtype=np.int32)
        stats = np.zeros((len(blocks), 3))
        _check(self.L.tnqe_debug_select(self.h, len(blocks), _iptr(nblk), _iptr(n if len(n) else kept), _dptr(sv),
                                        int(chi), float(tau), _iptr(kept), _dptr(stats)), self.h)
        return kept[:len(n)], stats

    def solve_batch(self, uploaded, chis, **kw):
        """Solve several uploaded subspaces; chis[s] is subspace s's bond cap."""
        n = len(uploaded)
        o = (_Opts * n)(*[options(chi=int(ch), **kw) for ch in chis])
        Hs = [np.zeros((u.M, u.M)) for u in uploaded]
        Ss = [np.zeros((u.M, u.M)) for u in uploaded]
        E = np.zeros(n)
        reps = (_Report * n)()
        handles = (C.c_void_p * n)(*[u.handle.value for u in uploaded])
        hp = (C.POINTER(C.c_double) * n)(*[_dptr(x) for x in Hs])
        sp = (C.POINTER(C.c_double) * n)(*[_dptr(x) for x in Ss])
        _check(self.L.tnqe_solve_batch(self.h, n, handles, o, hp, sp, _dptr(E), reps), self.h)
        return Hs, Ss, E, [report_dict(r) for r in reps]


class Uploaded:
    """Problem data resident in device memory."""

    def __init__(self, ctx, handle, M):
        self.ctx, self.handle, self.M = ctx, handle, M

    def solve(self, **kw):
        o = options(**kw)
        M = self.M
        H = np.zeros((M, M))
        S = np.zeros((M, M))
        E = np.zeros(1)
        c = np.zeros(M)
        r = _Report()
        _check(self.ctx.L.tnqe_solve(self.ctx.h, self.handle, C.byref(o), _dptr(H), _dptr(S), _dptr(E), _dptr(c),
                                     C.byref(r)), self.ctx.h)
        return H, S, float(E[0]), c, report_dict(r)

    def free(self):
        if self.handle:
            self.ctx.L.tnqe_problem_free(self.handle)
            self.handle = None


# ------------------------------------------------------------- host diagnostics
def debug_givens(W):
    W = np.ascontiguousarray(W, dtype=np.float64)
    N = W.shape[0]
    K = N * (N - 1) // 2
    pos = np.zeros(max(K, 1), dtype=np.int32)
    th = np.zeros(max(K, 1))
    det = np.zeros(1, dtype=np.int32)
    _check(lib().tnqe_debug_givens(N, _dptr(W), _iptr(pos), _dptr(th), _iptr(det)))
    return list(zip(pos[:K].tolist(), th[:K].tolist())), int(det[0])


def debug_gate(theta):
    out = np.zeros(256)
    _check(lib().tnqe_debug_gate(float(theta), _dptr(out)))
    return out.reshape(16, 16)


def debug_host_pool(workers, jobs):
    """Back-to-back parallel loops on the library's host worker pool; returns
    the number of item calls (raises if an item ran zero or several times)."""
    calls = C.c_int64(0)
    _check(lib().tnqe_debug_host_pool(int(workers), int(jobs), C.byref(calls)))
    return calls.value


def debug_mpo_dense(h, g):
    h = np.ascontiguousarray(h, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    N = h.shape[0]
    D = 4 ** N
    H = np.zeros((D, D))
    I = np.zeros((D, D))
    mb = np.zeros(1, dtype=np.int32)
    _check(lib().tnqe_debug_mpo_dense(N, _dptr(h), _dptr(g), _dptr(H), _dptr(I), _iptr(mb)))
    return H, I, int(mb[0])
