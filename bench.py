"""Throughput of the subspace pencil (H, S) and its lowest eigenvalue on one MI355X.

Workload: N = 24 spatial orbitals, chi = 256, M = 16 MPS (136 unique pairs),
12 + 12 electrons, 24 Cholesky vectors: the seeded synthetic stand-in for the
paper's molecular workloads (integrals, rotations and MPS drawn by
tnqe_synth from fixed seeds).  One step = one
complete solve (Givens networks with SVD truncation for the 120 off-diagonal
pairs, environment sweeps for all 136 pairs, the 16 x 16 generalized
eigenproblem) with the problem data already resident in HBM.

Prints one JSON line: metric, value (H/S elements per second), roofline of the
dominant kernel, and the FP64 CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "H/S elements/s (N=24, chi=256); mixed vs FP64 speedup at |dE|<=1e-6 Ha"
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


SVD_KERNELS = ["k_jacobi<%d>" % (4 * (k + 1)) for k in range(6)] + ["k_jacobi_global", "k_qr_blocks"] + [None] * 8
JACOBI_FAMILY = "k_jacobi<E>"
KERNEL_SOURCE = {"k_jacobi": "kernels_svd.hip", "k_env": "kernels_env.hip", "k_mix": "kernels_env.hip", "k_qr": "kernels_gate.hip"}
TRAFFIC_FILE = os.path.join(HERE, "profiles", "traffic.md")
ENV_KERNELS = ["k_env_g1", "k_mix", "k_env_gd", "k_env_g2", "k_env_final", None, None, None]
MACHINE_BALANCE = PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)   # flop per byte


def roofline(rep):
    """Roofline of the kernel with the most device time in the solve (the
    register Jacobi kernel taken over all its instantiations).

    Every launch is timed by the library with HIP events on the stream it runs
    on; achieved = algorithmic work of its launches / their summed duration
    (= per-launch work / mean launch duration).  SVD kernels are FP64 vector
    arithmetic ("alu", peak 78.6 TFLOP/s); environment kernels are priced
    against HBM when their arithmetic intensity is below the FP64 machine
    balance, else against the FP64 peak.
    """
    cands = []
    # the register-resident Jacobi kernel counts as one kernel over its
    # instantiations k_jacobi<4> ... k_jacobi<24> (components per lane): a gate
    # step runs several of them side by side, and which one has the most time
    # changes from run to run
    fam = [k for k, name in enumerate(SVD_KERNELS) if name and name.startswith("k_jacobi<")]
    fam_launches = sum(rep["svd_kind_launches"][k] for k in fam)
    if fam_launches > 0:
        cands.append((sum(rep["svd_kind_ms"][k] for k in fam), JACOBI_FAMILY,
                      sum(rep["svd_kind_flops"][k] for k in fam), None, fam_launches))
    for k, name in enumerate(SVD_KERNELS):
        if name and k not in fam and rep["svd_kind_launches"][k] > 0:
            cands.append((rep["svd_kind_ms"][k], name, rep["svd_kind_flops"][k], None, rep["svd_kind_launches"][k]))
    for k, name in enumerate(ENV_KERNELS):
        if name and rep["env_kind_launches"][k] > 0:
            cands.append((rep["env_kind_ms"][k], name, rep["env_kind_flops"][k], rep["env_kind_bytes"][k],
                          rep["env_kind_launches"][k]))
    if not cands:
        return None
    ms, name, flops, nbytes, launches = max(cands)
    sec = ms * 1e-3
    out = {"kernel": name, "launches": launches, "avg_launch_us": ms * 1e3 / launches}
    traffic = measured_traffic(name)
    if nbytes is None or (nbytes > 0 and flops / nbytes >= MACHINE_BALANCE):
        out.update({"bound": "alu", "achieved": flops / sec / 1e12, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                    "work_per_launch": flops / launches, "work_unit": "flop"})
    else:
        out.update({"bound": "hbm", "achieved": nbytes / sec / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "work_per_launch": nbytes / launches, "work_unit": "byte"})
    out["frac"] = out["achieved"] / out["peak"]
    out["traffic"] = traffic["bytes_per_launch"] if traffic else None
    out["traffic_unit"] = "bytes per launch (HBM, FETCH_SIZE + WRITE_SIZE scaled by a copy kernel)"
    out["traffic_detail"] = traffic
    return out


def kernel_breakdown(rep):
    """Device time, launches and algorithmic rates of every timed kernel kind."""
    out = []
    for k, name in enumerate(SVD_KERNELS):
        if name and rep["svd_kind_launches"][k] > 0:
            ms, fl = rep["svd_kind_ms"][k], rep["svd_kind_flops"][k]
            out.append({"kernel": name, "ms": ms, "launches": rep["svd_kind_launches"][k],
                        "tflops": fl / (ms * 1e-3) / 1e12 if ms > 0 else None})
    for k, name in enumerate(ENV_KERNELS):
        if name and rep["env_kind_launches"][k] > 0:
            ms, fl, by = rep["env_kind_ms"][k], rep["env_kind_flops"][k], rep["env_kind_bytes"][k]
            out.append({"kernel": name, "ms": ms, "launches": rep["env_kind_launches"][k],
                        "tflops": fl / (ms * 1e-3) / 1e12 if ms > 0 else None,
                        "gbs": by / (ms * 1e-3) / 1e9 if ms > 0 else None})
    return sorted(out, key=lambda x: -x["ms"])


def source_digest(kernel):
    import hashlib
    for prefix, f in KERNEL_SOURCE.items():
        if kernel.startswith(prefix):
            with open(os.path.join(HERE, "paper_2404_10223_amd", "csrc", f), "rb") as fh:
                return hashlib.sha256(fh.read()).hexdigest()
    return None


def measured_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    covers this kernel and its source file is unchanged since (else None)."""
    try:
        text = open(TRAFFIC_FILE).read()
        blob = text.split("```json", 1)[1].split("```", 1)[0]
        rec = json.loads(blob)
    except (OSError, IndexError, ValueError):
        return None
    entry = rec.get("kernels", {}).get(kernel)
    if not entry or entry.get("source_sha256") != source_digest(kernel):
        return None
    return {"bytes_per_launch": entry["fetch_bytes_per_launch"] + entry["write_bytes_per_launch"],
            "fetch_bytes_per_launch": entry["fetch_bytes_per_launch"],
            "write_bytes_per_launch": entry["write_bytes_per_launch"], "source": "profiles/traffic.md"}


def copy_calibration(nbytes=1 << 30):
    """A plain device copy of known size: the reference for scaling the
    FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    torch.cuda.synchronize()
    b = a.clone()
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "ok": bool(b[0].item() == 1)}))


def _host_info():
    """Host cores this process may use, CPU model, BLAS library and threads."""
    cores = len(os.sched_getaffinity(0))
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas = []
    try:
        from threadpoolctl import threadpool_info
        blas = [{"api": x.get("user_api"), "library": x.get("internal_api"), "threads": x.get("num_threads")}
                for x in threadpool_info()]
    except Exception:
        pass
    return cores, model, blas


def cpu_baseline(prob, diag=(0, 0), offd=(0, 1)):
    """The FP64 oracle on the same scope as the GPU's timed region, on a
    bounded sample: the MPO of basis i (built once per basis), one diagonal
    pair (environment sweep) and one off-diagonal pair (centre moves, gates
    with SVD truncation, environment sweep), and the eigensolve.  The job's
    time is extrapolated per part: M MPO builds, M diagonal and M (M - 1) / 2
    off-diagonal elements, one eigensolve.  A plain reference, not a tuned
    CPU code."""
    import numpy as np
    from oracle import gep as ogep
    from oracle.mpo import build_mpo, expectation
    from oracle.subspace import rotate_integrals, rotate_ket
    cores, model, blas = _host_info()
    i = diag[0]
    bi = prob.mps[i]
    t0 = time.perf_counter()
    hi, Li = rotate_integrals(prob.h, prob.L, bi.U)
    W = build_mpo(hi, np.einsum("kpq,krs->pqrs", Li, Li))
    t_mpo = time.perf_counter() - t0
    t0 = time.perf_counter()
    expectation(W, bi.sites, bi.bond_qn, bi.sites, bi.bond_qn)
    t_diag = time.perf_counter() - t0
    a, b = offd
    assert a == i
    bj = prob.mps[b]
    t0 = time.perf_counter()
    ket, kqn, _ = rotate_ket(bj.sites, bj.bond_qn, bi.U.T @ bj.U, prob.chi)
    t_gates = time.perf_counter() - t0
    t0 = time.perf_counter()
    expectation(W, bi.sites, bi.bond_qn, ket, kqn)
    t_env = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    A = rng.normal(size=(prob.M, prob.M))
    t0 = time.perf_counter()
    ogep.solve_projection(A + A.T, A @ A.T + np.eye(prob.M))
    t_gep = time.perf_counter() - t0
    M = prob.M
    n_off, n_pairs = M * (M - 1) // 2, M * (M + 1) // 2
    total = M * t_mpo + M * t_diag + n_off * (t_gates + t_env) + t_gep
    sample_s = t_mpo + t_diag + t_gates + t_env + t_gep
    return {"value": n_pairs / total, "unit": "elements/s", "cores": cores, "kind": "oracle",
            "cpu_model": model, "blas": blas,
            "sample": f"N={prob.N}, chi={prob.chi}, M={M}: MPO of basis {i} {t_mpo:.1f} s, diagonal pair {diag} "
                      f"environment sweep {t_diag:.1f} s, off-diagonal pair {offd} Givens network with SVD "
                      f"truncation {t_gates:.1f} s + environment sweep {t_env:.1f} s, eigensolve {t_gep * 1e3:.2f} ms "
                      f"({sample_s:.0f} s in all); extrapolated to {M} MPO builds, {M} diagonal and {n_off} "
                      f"off-diagonal elements: {total:.0f} s for the {n_pairs} elements",
            "extrapolated_job_s": total}


def cpu_single_thread_small():
    """The oracle's whole pencil for the N = 7, chi = 16, M = 4 workload on one
    BLAS thread (elements/s)."""
    import tnqe_synth as synth
    from oracle.subspace import subspace
    prob = synth.make_config(2)
    from threadpoolctl import threadpool_limits
    t0 = time.perf_counter()
    with threadpool_limits(limits=1):
        subspace(prob)
    dt = time.perf_counter() - t0
    n = prob.M * (prob.M + 1) // 2
    return {"value": n / dt, "unit": "elements/s", "threads": 1,
            "workload": "N=7, chi=16, M=4 (10 elements), whole pencil with sector-FCI H"}


def batch_line(ctx, steps):
    """The batched workload: 64 independent subspaces (N in 8..16, chi in
    {16, 32, 64, 128}, M in 2..8), inputs resident on the device, in one
    tnqe_solve_batch call: concurrent worker contexts (the library's default)
    against one subspace after another, FP64 and mixed precision."""
    import numpy as np
    import torch
    import tnqe_synth as synth
    probs = synth.make_batch()
    ups = [ctx.upload(p) for p in probs]
    n_el = sum(p.M * (p.M + 1) // 2 for p in probs)
    chis = [p.chi for p in probs]
    out = {"workload": "64 subspaces, N ~ U{8..16}, chi ~ U{16,32,64,128}, M ~ U{2..8}, half filling, K = N",
           "elements": n_el}
    try:
        def timed(**kw):
            ctx.solve_batch(ups, chis, autotune=True, **kw)          # warm-up (and tuning)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(max(1, steps)):
                res = ctx.solve_batch(ups, chis, autotune=True, **kw)
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) / max(1, steps), res
        t_seq, (Hs, Ss, Es, _) = timed(workers=1)
        t_par, _ = timed()
        t_mix, (Hm, Sm, Em, _) = timed(precision="mixed")
        dE = float(np.max(np.abs(np.asarray(Em) - np.asarray(Es))))
        out.update({"fp64_concurrent": {"value": n_el / t_par, "ms": t_par * 1e3},
                    "fp64_one_after_another": {"value": n_el / t_seq, "ms": t_seq * 1e3},
                    "mixed_concurrent": {"value": n_el / t_mix, "ms": t_mix * 1e3, "max_dE_Ha": dE,
                                         "valid": dE <= 1e-6},
                    "unit": "elements/s"})
        log(f"  batch: concurrent {n_el / t_par:.1f} el/s, one after another {n_el / t_seq:.1f} el/s, "
            f"mixed {n_el / t_mix:.1f} el/s (max dE {dE:.1e})")
    finally:
        for u in ups:
            u.free()
    return out


def sweep_line(ctx, steps, with_cpu):
    """One generalized-sweep step (Alg. A.1: expanded pencil of one state at
    one bond, discard, expanded root, parameter update, Givens angle search,
    truncation, one single-site mitigation round of App. A4) at N = 7 (chi = 16, state 3, sites 2-3) and N = 12 (chi = 64,
    state 0, sites 1-2), the current pencil from the library; the oracle's
    time for the N = 7 step when the CPU leg runs."""
    import torch
    import tnqe_synth as synth
    out = {}
    for k, i, p in ((2, 3, 2), (3, 0, 1)):
        prob = synth.make_config(k)
        H, S, E, c, _ = ctx.subspace(prob, chi=prob.chi)
        ctx.sweep_step(prob, H, S, i, p, rotation="givens", nreps=1, chi=prob.chi)      # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(max(1, steps)):
            res, _, _, rep = ctx.sweep_step(prob, H, S, i, p, rotation="givens", nreps=1, chi=prob.chi)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / max(1, steps) * 1e3
        d = {"workload": f"N={prob.N}, chi={prob.chi}, M={prob.M}, state {i}, sites {p}-{p + 1}, Givens rotation, "
                         "one single-site mitigation round",
             "ms_per_step": ms, "one_hot_states": res["n_onehot"], "columns": res["n_columns"],
             "kept_columns": res["n_kept"], "E_old": res["E_old"], "E1": res["E1"], "E_new": res["E_new"],
             "theta": res["theta"],
             "xi_none": res["xi_none"], "xi": res["xi"], "pencil_networks_ms": rep["t_gates_ms"],
             "pencil_contractions_ms": rep["t_env_ms"], "discard_and_eigensolve_ms": rep["t_gep_ms"],
             "step_ms_in_library": rep["t_total_ms"]}
        if with_cpu and k == 2:
            from oracle import sweep as osweep
            t1 = time.perf_counter()
            osweep.sweep_step(prob, H, S, i, p, rotation="givens", nreps=1)
            d["cpu_oracle_ms"] = (time.perf_counter() - t1) * 1e3
        out[f"N{prob.N}"] = d
        log(f"  sweep step N={prob.N}: {ms:.1f} ms (E_old {res['E_old']:.6f} -> E1 {res['E1']:.6f}, "
            f"theta {res['theta']:.4f})")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--rotations", choices=["expm", "perm", "identity"], default="expm",
                    help="orbital rotations of the MPS: random (TNQE, the headline workload), "
                         "permutations (fermionic-swap networks, TNQE-F) or none (LC-MPS)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--sweep-only", action="store_true",
                    help="only the generalized-sweep-step line (for profiling it); prints that line")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.sweep_only:
        import paper_2404_10223_amd as T
        ctx = T.Context(0)
        print(json.dumps({"sweep_step": sweep_line(ctx, args.steps, not args.no_cpu)}))
        ctx.close()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1 (the pairs would be "
                                   "sharded over GPUs by estimated cost; no multi-GPU path is built)"}))
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2404_10223_amd as T
    import tnqe_synth as synth

    prob = synth.make_config(5, args.rotations)
    ctx = T.Context(0)
    torch.cuda.synchronize()
    t_up = time.perf_counter()
    up = ctx.upload(prob)
    torch.cuda.synchronize()
    upload_s = time.perf_counter() - t_up
    n_pairs = prob.M * (prob.M + 1) // 2

    def run(steps, precision):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = None
        for _ in range(steps):
            out = up.solve(chi=prob.chi, precision=precision, autotune=True)
            log(f"  step {precision}: {out[4]['t_total_ms']:.1f} ms")
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, out

    # the first warm-up solve tunes the environment tile shapes (cached on
    # disk); the timed solves only look them up
    tune_ms = 0.0
    for _ in range(max(1, args.warmup)):
        tune_ms += run(1, "fp64")[1][4]["t_tune_ms"]
    t64, (H, S, E, c, rep) = run(args.steps, "fp64")
    value = n_pairs / t64
    mixed = None
    if not args.no_mixed:
        # every reduced-precision mode on the same GPU: time per solve, the
        # eigenvalue error against the FP64 path, and the speedup where the
        # error is within 1e-6 Ha
        modes = {"mixed": "FP32 environments for the pairs whose rotated ket keeps <= 1e-6 of its squared norm "
                          "(the element and its rounding are bounded by the ket norm), FP64 elsewhere",
                 "fp32": "every pair in FP32 (storage and matrix cores)",
                 "fp32_shift": "every pair in FP32 on H - c N with c N_e = the FP64 H_00 (eigenvalue shifted back)",
                 "bf16x3": "every pair on BF16 matrix cores with hi/lo split operands (3 products), FP32 "
                           "accumulation, shifted operator",
                 "bf16": "every pair on BF16 matrix cores (operands rounded to BF16), FP32 accumulation, shifted "
                         "operator"}
        mixed = {}
        for name, what in modes.items():
            run(1, name)
            tm, (Hm, Sm, Em, cm, repm) = run(args.steps, name)
            dE = abs(Em - E)
            mixed[name] = {"precision": what, "fp32_pairs": repm["n_fp32_pairs"], "ms_per_step": tm * 1e3,
                           "dE_Ha": dE, "valid": dE <= 1e-6, "speedup_vs_fp64": (t64 / tm) if dE <= 1e-6 else None,
                           "env_ms": repm["t_env_ms"],
                           "max_rel_dH": float(np.max(np.abs(Hm - H) / np.maximum(np.abs(H), 1e-300))),
                           "max_rel_dS": float(np.max(np.abs(Sm - S) / np.maximum(np.abs(S), 1e-300)))}
            log(f"  {name}: dE {dE:.2e} Ha, {tm * 1e3:.1f} ms per solve")
    batch = None if args.no_batch else batch_line(ctx, args.steps)
    sweep = None if args.no_sweep else sweep_line(ctx, args.steps, not args.no_cpu)
    roof = roofline(rep)
    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(prob)
        cpu["single_thread_small"] = cpu_single_thread_small()
    line = {"metric": METRIC, "value": value, "unit": "elements/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": t64 * 1e3, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "N=24 orbitals, chi=256, M=16 MPS (136 pairs), 12+12 electrons, "
                                   "24 Cholesky vectors, FP64 path"
                                   + {"expm": "", "perm": ", orbital permutations (fermionic-swap networks)",
                                      "identity": ", no orbital rotations (LC-MPS)"}[args.rotations],
                       "N": prob.N, "chi": prob.chi, "M": prob.M,
                       "pairs": n_pairs, "parallelism": "single GPU"},
            "E": E, "report": {k: rep[k] for k in ("t_host_ms", "t_gates_ms", "t_env_ms", "t_gep_ms",
                                                   "max_discarded_weight_sum", "min_rel_gap", "max_bond",
                                                   "svd_kernel_ms", "svd_flops", "move_kernel_ms", "move_flops",
                                                   "move_launches", "t_moves_ms", "env_kernel_ms", "env_flops",
                                                   "alg_bytes")},
            "mixed": mixed, "autotune_ms": tune_ms, "batch": batch, "sweep_step": sweep, "roofline": roof,
            "kernels": kernel_breakdown(rep), "cpu_baseline": cpu,
            "pcie_inclusive": {"upload_ms": upload_s * 1e3, "value": n_pairs / (t64 + upload_s),
                               "note": "one host-to-HBM upload of the integrals and the 16 MPS (first upload of "
                                       "the process) added to one solve; not the headline value"}}
    up.free()
    ctx.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
