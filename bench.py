#!/usr/bin/env python
"""Helmholtz multigrid benchmark on one MI355X.

Workload: cubed-sphere C192 x 70 (221,184 columns, 15,482,880 unknowns),
synthetic SPD face-coupling operator (w_h = 1, w_v = 1000 graded with
exp(-k/20), delta ~ U[0.5, 1.5]), b ~ N(0, 1), 6-level V-cycle (2/2 block-Jacobi
sweeps, omega = 0.8, 4 coarse sweeps).

A step is one complete solve of H x = b to relative residual 1e-6 by
conjugate gradients in float64 preconditioned by one float32 V-cycle per
iteration (operator apply, smoothing with column tridiagonal solves,
residual + restriction, prolongation, coarse sweeps, float64 Krylov
updates), with b and x resident in HBM. `value` is solves per second, timed
with the library's kernel timing hook off. A second pass of the same steps
with the hook on gives the dominant kernel's duration (the roofline) and the
in-solve V-cycle time. Beside them: the float64-only solve on the same seed,
the V-cycle entry points, the set-up, the adjoint (backward) step, the
achievable bandwidth of plain streaming kernels, and the oracle on one host
core (a separate single-threaded process that runs while the GPU works; its
float64 solution to 1e-12 is what the GPU solutions' errors are measured
against).
"""
from __future__ import annotations

import os
import sys

# The CPU baseline times the oracle on one host core: its worker process pins
# the thread pools before NumPy is imported.
_WORKER = "--cpu-baseline-worker" in sys.argv
if _WORKER:
    for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[_v] = "1"

import argparse  # noqa: E402
import hashlib  # noqa: E402
import json  # noqa: E402
import platform  # noqa: E402
import subprocess  # noqa: E402
import tempfile  # noqa: E402
import time  # noqa: E402

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads  # noqa: E402

PEAK_HBM_GBS = 8000.0


def vcycle_words(L, n_pre, n_post, n_coarse):
    """Words per finest-level unknown that one V-cycle of this library's
    kernels moves.

    Per level: first sweep from zero 4 words (b, two column factors, x_new),
    further sweeps 7 (b, x, two face couplings, two factors, x_new), fused
    residual + restriction 6 + 1/4 (b, x, kh[2], kv, delta; coarse b), sweep
    with fused prolongation 7 + 1/4 (coarse x). Level l has 4^-l of the
    finest level's unknowns.
    """
    def smooth(n, first_zero):
        if n == 0:
            return 0.0
        return (4.0 if first_zero else 7.0) + 7.0 * (n - 1)

    total = 0.0
    for l in range(L - 1):
        words = smooth(n_pre, True)
        words += 6.25 if n_pre > 0 else 1.25
        if n_post > 0:
            words += 7.25 + 7.0 * (n_post - 1)
        else:
            words += 2.25
        total += words * 4.0 ** (-l)
    total += smooth(n_coarse, True) * 4.0 ** (-(L - 1))
    return total


# Words per unknown that the method itself must move, with the block-Jacobi
# step in the residual form of Eq. jacobi (x + omega Hz^-1 (b - H x)): a sweep
# reads b, x, the four coefficient arrays of H it needs (kh E and N, kv,
# delta) and the column factor and writes x_new (8 words; 4 from a zero
# guess); residual + restriction 6.25; the sweep that adds the prolongated
# correction 8.25. This is the count the roofline and the V-cycle fraction
# are quoted on; the kernels move fewer (see vcycle_words: the sweep is
# evaluated in a form that needs neither delta nor kv).
METHOD_SWEEP_WORDS = 8.0


def method_vcycle_words(L, n_pre, n_post, n_coarse):
    """Words per finest-level unknown of one V-cycle by the method's byte
    model (34.5 per level above the coarsest and 28 on it for 2/2/4 sweeps)."""
    def smooth(n):
        return 4.0 + METHOD_SWEEP_WORDS * (n - 1) if n > 0 else 0.0

    total = 0.0
    for l in range(L - 1):
        words = smooth(n_pre) + (6.25 if n_pre > 0 else 1.25)
        words += (8.25 + METHOD_SWEEP_WORDS * (n_post - 1)) if n_post > 0 else 2.25
        total += words * 4.0 ** (-l)
    return total + smooth(n_coarse) * 4.0 ** (-(L - 1))


def cg_bytes_per_unknown(vc_words, mixed, flexible):
    """Algorithmic bytes per unknown of one CG iteration (outer loop in float64).
    The x update rides with the p update, which reads p once for both."""
    apply_dot = 6 * 8                      # p, kh[2], kv, delta read; q written
    update = 2 * 8 + 8 + (4 if mixed else 0)   # r, q read; r (, r32) written
    vc = vc_words * (4 if mixed else 8)
    zsz = 4 if mixed else 8
    dot = 8 + zsz + (8 if flexible else 0)
    pupd = zsz + 8 + 8 + 8 + 8             # z, p, x read; p, x written
    return apply_dot + update + vc + dot + pupd


def bicgstab_bytes_per_unknown(vc_words, mixed):
    """Algorithmic bytes per unknown of one BiCGStab iteration (outer loop in
    float64): two preconditioner applications (float32 ones convert their
    input and output), two applies with a fused inner product, and the p, s
    and x/r updates."""
    precond = vc_words * (4 if mixed else 8) + (2 * (8 + 4) if mixed else 0)
    apply_dot = 6 * 8 + 8              # p_hat or s_hat, kh[2], kv, delta, dot partner; out
    p_upd = 3 * 8 + 8                  # r, v, p read; p written
    s_upd = 2 * 8 + 8                  # r, v read; s written
    xr_upd = 2 * 8 + 5 * 8 + 8         # x read+written; p_hat, s_hat, s, t, r0 read; r written
    return 2 * (precond + apply_dot) + p_upd + s_upd + xr_upd


def kernel_sources_hash():
    h = hashlib.sha256()
    for f in ("kernels.hpp", "helmholtz.hip"):
        h.update(open(os.path.join(ROOT, "paper_2002_00756_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(path):
    """HBM bytes per launch of the profiled kernel from the committed counter summary,
    or None if there is none or the kernel sources changed since it was taken."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip("# ").strip()] = v.strip()
    if vals.get("kernel sources sha256 prefix") != kernel_sources_hash():
        return None
    return float(vals["traffic bytes/dispatch"])


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline_worker(outdir):
    """Run in its own process (thread pools pinned to one thread before NumPy
    was imported): the float64 oracle's set-up, one apply, one V-cycle and a
    full MG-preconditioned CG solve at C12x10 (to 1e-8), C96x30 and C192x70
    (to 1e-6), each timed on the wall clock. The C192x70 solve is run on to
    1e-12; the time and iterate where its residual first reaches 1e-6 are the
    1e-6 solve (the iteration up to there is the same), and both that iterate
    and the 1e-12 solution are saved to `outdir` for the error of the GPU
    solutions. Prints one JSON object."""
    from oracle import helmholtz, krylov, mesh, multigrid
    pools = []
    try:
        from threadpoolctl import threadpool_info
        pools = [{"api": p.get("internal_api"), "threads": p.get("num_threads")}
                 for p in threadpool_info()]
    except Exception:  # pragma: no cover
        pass
    cases = []
    for w, rtol in ((workloads.C12x10, 1e-8), (workloads.C96x30, 1e-6),
                    (workloads.C192x70, 1e-6)):
        kh, kv, delta = workloads.workload_coefficients(w)
        b = workloads.rhs(w.N, w.nz)[0]
        t0 = time.perf_counter()
        levels, parents, childs = mesh.hierarchy(w.N, w.nlevels)
        hier = helmholtz.Hierarchy(levels, parents, childs, kh, kv, delta)
        t1 = time.perf_counter()
        hier.apply(0, b)
        t2 = time.perf_counter()
        multigrid.vcycle(hier, b)
        t3 = time.perf_counter()
        _log(f"cpu baseline {w.name}: set-up {t1 - t0:.2f} s, apply {t2 - t1:.2f} s, "
             f"V-cycle {t3 - t2:.2f} s")
        full = w.name == "C192x70"
        hit = {}

        def watch(it, x, rel, t_start=time.perf_counter()):
            if rel <= rtol and "t" not in hit:
                hit.update(t=time.perf_counter() - t_start, it=it, rel=rel)
                if full:
                    np.save(os.path.join(outdir, "x_1e-6.npy"), x)
            if full:
                _log(f"  oracle CG {w.name} iteration {it}: relres {rel:.3e}")

        res = krylov.solve(hier, b, rtol=1e-12 if full else rtol, maxiter=100, callback=watch)
        if full:
            np.save(os.path.join(outdir, "x_ref.npy"), res.x)
        cases.append({"workload": w.name, "unknowns": w.n, "levels": w.nlevels,
                      "setup_s": t1 - t0, "apply_s": t2 - t1, "vcycle_s": t3 - t2,
                      "rtol": rtol, "solve_s": hit["t"], "iters": hit["it"],
                      "relres": hit["rel"],
                      **({"iters_to_1e-12": res.iters, "relres_final": res.relres}
                         if full else {})})
    print(json.dumps({"cases": cases, "cpu_count": os.cpu_count(), "cpu_model": cpu_model(),
                      "thread_env": {v: os.environ.get(v) for v in
                                     ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS",
                                      "MKL_NUM_THREADS")},
                      "threadpools": pools}), flush=True)


def start_cpu_baseline():
    """Start the oracle worker (see cpu_baseline_worker) beside the GPU work."""
    outdir = tempfile.mkdtemp(prefix="hh_oracle_")
    env = dict(os.environ)
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[v] = "1"
    proc = subprocess.Popen([sys.executable, os.path.abspath(__file__),
                             "--cpu-baseline-worker", outdir],
                            stdout=subprocess.PIPE, env=env, text=True)
    return proc, outdir


def finish_cpu_baseline(proc, outdir):
    out, _ = proc.communicate()
    if proc.returncode != 0:
        raise RuntimeError(f"cpu baseline worker failed ({proc.returncode})")
    rep = json.loads(out.strip().splitlines()[-1])
    big = [c for c in rep["cases"] if c["workload"] == "C192x70"][0]
    sample = ("measured float64 oracle solves (NumPy, one thread) on the GPU host: "
              + "; ".join(f"{c['workload']}: {c['iters']} CG iterations to {c['rtol']:g} in "
                          f"{c['solve_s']:.2f} s (V-cycle {c['vcycle_s']:.2f} s, apply "
                          f"{c['apply_s']:.2f} s, set-up {c['setup_s']:.2f} s not counted)"
                          for c in rep["cases"])
              + "; value = 1 / the C192x70 solve time")
    base = {"value": 1.0 / big["solve_s"], "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": sample, "cpu_model": rep["cpu_model"], "cpu_count": rep["cpu_count"],
            "thread_env": rep["thread_env"], "threadpools": rep["threadpools"],
            "cases": rep["cases"]}
    x_ref = np.load(os.path.join(outdir, "x_ref.npy"))
    x_6 = np.load(os.path.join(outdir, "x_1e-6.npy"))
    for f in ("x_ref.npy", "x_1e-6.npy"):
        os.remove(os.path.join(outdir, f))
    os.rmdir(outdir)
    return base, x_ref, x_6, big


def stream_reference(torch, dev, lib, check, reps=10):
    """Achievable HBM bandwidth on this GPU, the yardstick beside the 8 TB/s
    peak: the library's own plain streaming kernels (read, write, copy and
    triad of 1 GiB float32 arrays, 16-byte accesses), best of `reps` launches
    each, timed with events on the stream they run on."""
    n = 1 << 28
    a = torch.full((n,), 1.0, dtype=torch.float32, device=dev)
    b = torch.full((n,), 2.0, dtype=torch.float32, device=dev)
    c = torch.empty_like(a)
    part = torch.empty(n // 4096 + 1, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    from paper_2002_00756_amd import _lib

    def launch(kind):
        dst = part if kind == _lib.BW_READ else c
        check(lib.helmholtz_bandwidth_kernel(kind, a.data_ptr(), b.data_ptr(), dst.data_ptr(),
                                             n, 3.0, stream.cuda_stream), "bandwidth_kernel")

    def best(kind, nbytes):
        launch(kind)
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            launch(kind)
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        return nbytes / (min(ms) * 1e-3) / 1e9

    out = {"read_GBps": best(_lib.BW_READ, 4 * n), "write_GBps": best(_lib.BW_WRITE, 4 * n),
           "copy_GBps": best(_lib.BW_COPY, 8 * n), "triad_GBps": best(_lib.BW_TRIAD, 12 * n)}
    ok = bool((c == 7.0).all()) and abs(float(part.double().sum()) - n) < 1e-3 * n
    del a, b, c, part
    torch.cuda.empty_cache()
    out.update(best_GBps=max(out.values()), checked=ok,
               kernels="helmholtz_bandwidth_kernel (hand-written HIP), 1 GiB float32 arrays")
    return out


def batch_leg(Operator, torch, dev, steps=2, warmup=1):
    """Largest single-GPU case: C384 x 70, batch of 4 right-hand sides sharing one
    operator, float32 7-level V-cycle in float64 CG to 1e-6; one step is a forward
    solve of all four plus the adjoint solve of all four and the face gradients."""
    w = workloads.C384x70
    kh, kv, delta = workloads.workload_coefficients(w)
    b = torch.from_numpy(workloads.rhs(w.N, w.nz, w.batch)).to(dev)
    g = torch.from_numpy(workloads.loss_weights(w.N, w.nz, w.batch)).to(dev)
    op = Operator(w.N, w.nz, kh, kv, delta, w.nlevels, precision="fp32", max_batch=w.batch,
                  device=dev)
    del kh, kv, delta

    def step():
        x = op.solve(b, rtol=1e-6)
        lam = op.solve(g, rtol=1e-6)
        op.face_grad(lam.x, x.x)
        return x, lam

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        x, lam = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) / steps * 1e3
    true = [float(torch.linalg.norm(b[i] - op.apply(x.x[i])) / torch.linalg.norm(b[i]))
            for i in range(w.batch)]
    return {
        "workload": f"{w.name} x batch {w.batch} ({w.n} unknowns per right-hand side)",
        "ms_per_fwd_adj_step": ms,
        "solves_per_s": 2 * w.batch * 1e3 / ms,
        "iters_fwd": x.iters, "iters_adj": lam.iters,
        "true_relres_max": max(true),
        "workspace_GB": op.workspace_bytes / 1e9,
    }


def solver_comparison(Operator, torch, dev, reps=5):
    """Pressure-solver configurations of the paper's Section 5.1 (Table 1) and
    the timestep-robustness study of Section 5.3 (Table 5), on the benchmark
    workload with the synthetic operator, float32 preconditioners inside
    float64 Krylov loops. Each entry: time per pressure solve (wall clock
    around the call, b and x in HBM), iterations (Krylov solvers), the true
    float64 relative residual reached, and GB/s of the byte model.

    Configurations: line relaxation = PreOnly with P_Jac(0.8, 10); Krylov(eps)
    = BiCGStab with P_Jac(1, 1); MG(L) = PreOnly with P_MG(L, 0.8, 2, 2), L =
    1..4; Krylov-MG(eps, 4) = BiCGStab with P_MG(4, 0.8, 2, 2); eps in {1e-2,
    1e-3, 1e-6}. Robustness: w_h = CFL_h^2 / 4 (the horizontal coupling
    relative to the mean of delta, which is 1) for CFL_h = 4, 6, 8, with
    MG(3), Kr2 = Krylov(1e-2) and Kr6 = Krylov(1e-6)."""
    w = workloads.C192x70
    n = w.n

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps * 1e3, r

    def run(coeffs, b, configs):
        bn = torch.linalg.norm(b)
        rows = []
        for name, L, prm, eps in configs:
            op = Operator(w.N, w.nz, *coeffs, L, *prm, precision="fp32",
                          cg="bicgstab" if eps else "standard", device=dev)
            if eps:
                ms, res = timed(lambda: op.solve(b, rtol=eps, maxiter=2000))
                x, iters = res.x, res.iters[0]
                gbs = bicgstab_bytes_per_unknown(vcycle_words(L, *prm[:3]), True) * iters * n
            else:
                ms, x = timed(lambda: op.vcycle(b))
                iters = None
                gbs = (vcycle_words(L, *prm[:3]) + 4.0) * 4 * n   # + layout conversion
            true = float(torch.linalg.norm(b - op.apply(x)) / bn)
            rows.append({"name": name, "ms": ms, "iters": iters, "relres": true,
                         "GBps": gbs / (ms * 1e-3) / 1e9})
            del op
        return rows

    MG = (2, 2, 4, 0.8)
    kh, kv, delta = workloads.workload_coefficients(w)
    coeffs = tuple(torch.from_numpy(a).to(dev) for a in (kh, kv, delta))
    b = torch.from_numpy(workloads.rhs(w.N, w.nz)[0]).to(dev)
    configs = [("line relaxation", 1, (2, 2, 10, 0.8), None)]
    configs += [(f"Krylov({e:g})", 1, (2, 2, 1, 1.0), e) for e in (1e-2, 1e-3, 1e-6)]
    configs += [(f"MG({L})", L, MG, None) for L in (1, 2, 3, 4)]
    configs += [(f"Krylov-MG({e:g},4)", 4, MG, e) for e in (1e-2, 1e-3, 1e-6)]
    table1 = run(coeffs, b, configs)
    del coeffs
    robust = []
    for cfl in (4, 6, 8):
        w_h = cfl * cfl / 4.0
        c = workloads.coefficients(w.N, w.nz, w_h, w.w_v, w.graded)
        coeffs = tuple(torch.from_numpy(a).to(dev) for a in c)
        rows = run(coeffs, b, [("MG(3)", 3, MG, None), ("Kr2", 1, (2, 2, 1, 1.0), 1e-2),
                               ("Kr6", 1, (2, 2, 1, 1.0), 1e-6)])
        robust.append({"CFL_h": cfl, "w_h": w_h, "solvers": rows})
        del coeffs
    return {"workload": f"{w.name} ({w.n} unknowns), float32 preconditioners, float64 Krylov",
            "table1": table1, "cfl_robustness": robust}


def nine_cell_leg(Operator, torch, dev, _lib, steps=10, warmup=2):
    """The 9-cell stencil of Section 3.5 on the benchmark shape (C192x70_9: the
    C192x70 operator plus couplings two levels apart, 1 % of the nearest
    ones): float32 V-cycle in float64 CG to 1e-6, the smoother dropping the
    k+-2 couplings from its column solve. Sweep and apply GB/s count the extra
    coefficient word (8 and 7 words per unknown)."""
    w = workloads.C192x70_9
    kh, kv, delta = workloads.workload_coefficients(w)
    kv2 = workloads.workload_kv2(w)
    op = Operator(w.N, w.nz, kh, kv, delta, w.nlevels, precision="fp32", device=dev, kv2=kv2)
    b = torch.from_numpy(workloads.rhs(w.N, w.nz)[0]).to(dev)
    for _ in range(warmup):
        op.solve(b, rtol=1e-6)
    torch.cuda.synchronize()
    op.profile(True)
    t = time.perf_counter()
    for _ in range(steps):
        res = op.solve(b, rtol=1e-6)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) / steps * 1e3
    sw_ms, sw_n, sw_b = op.profile_read(_lib.PROF_SWEEP_FINE)
    ap_ms, ap_n, ap_b = op.profile_read(_lib.PROF_APPLY_FINE)
    op.profile(False)
    true = float(torch.linalg.norm(b - op.apply(res.x)) / torch.linalg.norm(b))
    b32 = b.float()
    for _ in range(3):
        op.vcycle_f32(b32)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(20):
        op.vcycle_f32(b32)
    torch.cuda.synchronize()
    vc_ms = (time.perf_counter() - t) / 20 * 1e3
    return {
        "workload": f"{w.name} ({w.n} unknowns, w_v2 = {w.w_v2})",
        "solves_per_s": 1e3 / ms, "ms_per_solve": ms, "iters": res.iters[0],
        "true_relres": true, "vcycle_f32_ms": vc_ms,
        "sweep_fine_us": sw_ms / max(sw_n, 1) * 1e3,
        "sweep_fine_GBps": sw_b / (sw_ms * 1e-3) / 1e9 if sw_n else None,
        "apply_fine_GBps": ap_b / (ap_ms * 1e-3) / 1e9 if ap_n else None,
    }


def weighted_leg(Operator, torch, dev, steps=5, warmup=1):
    """The non-symmetric operator H = delta + diag(s) L on the benchmark shape
    (C192x70 coefficients, s ~ U[0.5, 1.5], the role of 1/rho*): BiCGStab with
    one float32 6-level V-cycle per preconditioner application, to 1e-6; the
    forward solve alone, and a gradient step (forward solve, adjoint solve with
    H^T and the transposed V-cycle, weighted face gradients)."""
    w = workloads.C192x70
    kh, kv, delta = workloads.workload_coefficients(w)
    sw = workloads.row_weights(w.N, w.nz)
    op = Operator(w.N, w.nz, kh, kv, delta, w.nlevels, precision="fp32", cg="bicgstab",
                  device=dev, s=sw)
    b = torch.from_numpy(workloads.rhs(w.N, w.nz)[0]).to(dev)
    g = torch.from_numpy(workloads.loss_weights(w.N, w.nz)[0]).to(dev)
    for _ in range(warmup):
        op.solve(b, rtol=1e-6)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        res = op.solve(b, rtol=1e-6)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) / steps * 1e3
    t = time.perf_counter()
    for _ in range(steps):
        xf = op.solve(b, rtol=1e-6)
        lam = op.solve_adjoint(g, rtol=1e-6)
        op.face_grad(lam.x, xf.x)
    torch.cuda.synchronize()
    step_ms = (time.perf_counter() - t) / steps * 1e3
    bn, gn = torch.linalg.norm(b), torch.linalg.norm(g)
    n = w.n
    gbs = bicgstab_bytes_per_unknown(vcycle_words(w.nlevels, 2, 2, 4), True) * res.iters[0] * n
    return {
        "workload": f"{w.name} coefficients with row weights s ~ U[0.5, 1.5] ({n} unknowns)",
        "solver": "BiCGStab + float32 MG(6) V-cycle, rtol 1e-6",
        "solves_per_s": 1e3 / ms, "ms_per_solve": ms, "iters": res.iters[0],
        "true_relres": float(torch.linalg.norm(b - op.apply(res.x)) / bn),
        "GBps": gbs / (ms * 1e-3) / 1e9,
        "adjoint_iters": lam.iters[0],
        "adjoint_true_relres": float(torch.linalg.norm(g - op.apply_adjoint(lam.x)) / gn),
        "fwd_adj_grad_step_ms": step_ms,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="C192x70", choices=sorted(workloads.ALL))
    ap.add_argument("--rtol", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch-leg", action="store_true",
                    help="skip the C384x70 batch-of-4 forward+adjoint measurement")
    ap.add_argument("--cg", default="standard", choices=["standard", "flexible"])
    ap.add_argument("--no-weighted", action="store_true",
                    help="skip the non-symmetric (row-weighted) operator measurement")
    ap.add_argument("--no-nine-cell", action="store_true",
                    help="skip the 9-cell stencil measurement")
    ap.add_argument("--no-solver-comparison", action="store_true",
                    help="skip the pressure-solver configurations of Section 5.1 and the "
                         "CFL robustness study")
    ap.add_argument("--probe", action="store_true",
                    help="for counter runs: a few solves (of the workload's whole batch) plus "
                         "a 1 GiB device copy of known size, no JSON")
    ap.add_argument("--cpu-baseline-worker", metavar="OUTDIR", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_baseline_worker:
        cpu_baseline_worker(args.cpu_baseline_worker)
        return
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(it has no multi-GPU path).", file=sys.stderr)
        sys.exit(2)

    w = workloads.ALL[args.workload]
    baseline = None
    if not args.no_cpu_baseline and not args.probe and args.workload == "C192x70":
        baseline = start_cpu_baseline()

    import torch
    from paper_2002_00756_amd import Operator, _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2002_00756_amd import build
        build.build()
    lib = _lib.load()

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    kh, kv, delta = workloads.workload_coefficients(w)
    b_np = workloads.rhs(w.N, w.nz)[0]
    prm = dict(n_pre=2, n_post=2, n_coarse=4, omega=0.8)

    # --- set-up (mesh tables, coarse operators, factors, float32 copies) ---
    kh_d = torch.from_numpy(kh).to(dev)
    kv_d = torch.from_numpy(kv).to(dev)
    dl_d = torch.from_numpy(delta).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op32 = Operator(w.N, w.nz, kh_d, kv_d, dl_d, w.nlevels, precision="fp32", cg=args.cg,
                    device=dev, **prm)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    op64 = Operator(w.N, w.nz, kh_d, kv_d, dl_d, w.nlevels, precision="fp64", cg="standard",
                    device=dev, **prm)
    b = torch.from_numpy(b_np).to(dev)
    x = torch.empty_like(b)
    stream = torch.cuda.current_stream(dev)

    def timed_solves(op, steps, warmup, hook=False):
        """Mean time of `steps` solves after `warmup` untimed ones, bracketed by
        device synchronisations. With `hook` the library's kernel timing hook
        records the timed solves' profiled launches."""
        for _ in range(warmup):
            op.solve(b, rtol=args.rtol, out=x)
        torch.cuda.synchronize()
        if hook:
            op.profile(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        its = []
        e0.record(stream)
        t = time.perf_counter()
        for _ in range(steps):
            res = op.solve(b, rtol=args.rtol, out=x)
            its.append(res.iters[0])
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        return e0.elapsed_time(e1) / steps, wall / steps * 1e3, its, res

    if args.probe:
        if w.batch > 1:
            # the workload's batch of right-hand sides through one handle
            del op32, op64
            torch.cuda.empty_cache()
            opb = Operator(w.N, w.nz, kh_d, kv_d, dl_d, w.nlevels, precision="fp32",
                           cg=args.cg, max_batch=w.batch, device=dev, **prm)
            bb = torch.from_numpy(workloads.rhs(w.N, w.nz, w.batch)).to(dev)
            for _ in range(max(args.steps, 1)):
                opb.solve(bb, rtol=args.rtol)
        else:
            for _ in range(max(args.steps, 1)):
                op32.solve(b, rtol=args.rtol, out=x)
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)          # reads and writes exactly 1 GiB each
        torch.cuda.synchronize()
        print("probe done", flush=True)
        return

    # --- the metric: mixed-precision solves, timing hook off ----------------
    ms32, wall32, its32, res32 = timed_solves(op32, args.steps, args.warmup)
    x32 = x.clone()
    true32 = float(torch.linalg.norm(b - op64.apply(x32)) / torch.linalg.norm(b))
    # --- float64-only path on the same seed ----------------------------------
    ms64, wall64, its64, res64 = timed_solves(op64, args.steps, args.warmup)
    x64 = x.clone()
    true64 = float(torch.linalg.norm(b - op64.apply(x64)) / torch.linalg.norm(b))

    # --- the same steps again with the kernel timing hook on -----------------
    # (dominant kernel, float64 apply and the whole in-solve V-cycle)
    hms32, _, _, _ = timed_solves(op32, args.steps, 2, hook=True)
    sweep_ms, sweep_n, sweep_kbytes = op32.profile_read(_lib.PROF_SWEEP_FINE)
    vc32_ms, vc32_n, vc32_kbytes = op32.profile_read(_lib.PROF_VCYCLE)
    op32.profile(False)
    hms64, _, _, _ = timed_solves(op64, args.steps, 2, hook=True)
    sw64_ms, sw64_n, sw64_kbytes = op64.profile_read(_lib.PROF_SWEEP_FINE)
    ap_ms, ap_n, ap_bytes = op64.profile_read(_lib.PROF_APPLY_FINE)
    vc64_ms_in, vc64_n, vc64_kbytes = op64.profile_read(_lib.PROF_VCYCLE)
    op64.profile(False)

    # reference solution on the GPU (float64 to 1e-12), used when the oracle's is absent
    xref_gpu = op64.solve(b, rtol=1e-12).x

    # --- V-cycle entry points (ABI layout in and out) ------------------------
    n = w.n
    words = vcycle_words(w.nlevels, prm["n_pre"], prm["n_post"], prm["n_coarse"])
    mwords = method_vcycle_words(w.nlevels, prm["n_pre"], prm["n_post"], prm["n_coarse"])

    def time_vcycle(fn, arg, reps=20):
        for _ in range(3):
            fn(arg)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn(arg)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    b32 = b.float()
    vce32_ms = time_vcycle(op32.vcycle_f32, b32)
    vce64_ms = time_vcycle(op64.vcycle, b)
    conv_words = 4.0   # the entry points convert b and x between the ABI and tiled layouts

    # --- adjoint step: forward solve + adjoint solve + face gradients ---------
    g = torch.from_numpy(workloads.loss_weights(w.N, w.nz)[0]).to(dev)
    torch.cuda.synchronize()
    t = time.perf_counter()
    reps_adj = max(1, min(3, args.steps))
    for _ in range(reps_adj):
        xf = op32.solve(b, rtol=args.rtol).x
        lam = op32.solve(g, rtol=args.rtol).x
        op32.face_grad(lam, xf)
    torch.cuda.synchronize()
    adj_ms = (time.perf_counter() - t) / reps_adj * 1e3

    # --- the differentiable solve: loss = g . x, forward + backward ----------
    # (the first call builds the operator; later ones take it from the pool
    # and replace its coefficients)
    from paper_2002_00756_amd import autograd as hh_autograd, helmholtz_solve
    leaves = [t_.clone().requires_grad_(True) for t_ in (kh_d, kv_d, dl_d)]

    def diff_step():
        xs = helmholtz_solve(b, *leaves, N=w.N, nz=w.nz, nlevels=w.nlevels,
                             precision="fp32", rtol=args.rtol, **prm)
        (g * xs).sum().backward()

    hh_autograd.clear_operator_pool()
    torch.cuda.synchronize()
    t = time.perf_counter()
    diff_step()
    torch.cuda.synchronize()
    diff_first_ms = (time.perf_counter() - t) * 1e3
    t = time.perf_counter()
    for _ in range(reps_adj):
        diff_step()
    torch.cuda.synchronize()
    diff_ms = (time.perf_counter() - t) / reps_adj * 1e3
    del leaves
    hh_autograd.clear_operator_pool()

    ref = stream_reference(torch, dev, lib, _lib.check)
    stream_gbs = ref["best_GBps"]

    # --- dominant kernel: fine-level float32 smoothing sweep -----------------
    sweep_avg_ms = sweep_ms / max(sweep_n, 1)
    sweep_method_bytes = METHOD_SWEEP_WORDS * 4 * n
    achieved = sweep_method_bytes / (sweep_avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(os.path.join(ROOT, "profiles", "traffic_sweep_f32_C192x70.txt"))

    def vc_stats(ms, cnt, kbytes, word):
        avg = ms / max(cnt, 1)
        return {"ms": avg, "count": cnt,
                "GBps": mwords * word * n / (avg * 1e-3) / 1e9,
                "frac": mwords * word * n / (avg * 1e-3) / 1e9 / PEAK_HBM_GBS,
                "GBps_kernel_words": kbytes / max(cnt, 1) / (avg * 1e-3) / 1e9}

    per_iter32 = cg_bytes_per_unknown(words, True, args.cg == "flexible")
    per_iter64 = cg_bytes_per_unknown(words, False, False)
    it32 = float(np.mean(its32))
    it64 = float(np.mean(its64))
    out = {
        "metric": "Helmholtz solves/s (FP32-MG preconditioned FP64 CG to rel res 1e-6)",
        "value": 1e3 / ms32,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 V-cycle + f64 CG",
        "data": "synthetic",
        "config": {
            "workload": f"{w.name} cubed sphere ({w.ncol} columns x {w.nz} levels, "
                        f"{w.n} unknowns), w_h={w.w_h}, w_v={w.w_v}"
                        f"{' graded exp(-k/20)' if w.graded else ''}",
            "levels": w.nlevels, "n_pre": 2, "n_post": 2, "n_coarse": 4, "omega": 0.8,
            "rtol": args.rtol, "cg": args.cg, "batch": 1,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_sweep<float> plain mode, finest level",
            "achieved": achieved,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": sweep_method_bytes,
            "words_per_unknown": METHOD_SWEEP_WORDS,
            "kernel_words_per_unknown": 7.0,
            "achieved_kernel_words": sweep_kbytes / max(sweep_n, 1) / (sweep_avg_ms * 1e-3) / 1e9,
            "frac_of_stream": achieved / stream_gbs,
            "avg_launch_us": sweep_avg_ms * 1e3,
            "launches": sweep_n,
            "timed_in": "second pass of the timed solves with the library's event hook on",
        },
        "fp32_mg": {
            "solves_per_s": 1e3 / ms32, "ms_per_solve": ms32, "host_wall_ms": wall32,
            "ms_per_solve_hook_on": hms32,
            "iters": it32, "true_relres": true32,
            "cg_GBps": it32 * per_iter32 * n / (ms32 * 1e-3) / 1e9,
        },
        "fp64_mg": {
            "solves_per_s": 1e3 / ms64, "ms_per_solve": ms64, "host_wall_ms": wall64,
            "ms_per_solve_hook_on": hms64,
            "iters": it64, "true_relres": true64,
            "cg_GBps": it64 * per_iter64 * n / (ms64 * 1e-3) / 1e9,
            "sweep_fine_GBps": METHOD_SWEEP_WORDS * 8 * n / (sw64_ms / max(sw64_n, 1) * 1e-3)
            / 1e9 if sw64_n else None,
            "apply_fine_GBps": (ap_bytes / max(ap_n, 1)) / (ap_ms / max(ap_n, 1) * 1e-3) / 1e9
            if ap_n else None,
        },
        "speedup_fp32mg_vs_fp64": ms64 / ms32,
        "vcycle_in_solve": {
            "words_per_unknown": mwords, "kernel_words_per_unknown": words,
            "fp32": vc_stats(vc32_ms, vc32_n, vc32_kbytes, 4),
            "fp64": vc_stats(vc64_ms_in, vc64_n, vc64_kbytes, 8),
            "note": "device time of each whole V-cycle inside the timed solves (event pair "
                    "around all its launches, gaps included)",
        },
        "vcycle_entry_points": {
            "fp32_ms": vce32_ms, "fp64_ms": vce64_ms,
            "fp32_GBps": (mwords + conv_words) * 4 * n / (vce32_ms * 1e-3) / 1e9,
            "fp64_GBps": (mwords + conv_words) * 8 * n / (vce64_ms * 1e-3) / 1e9,
            "note": "helmholtz_vcycle_f32 / helmholtz_vcycle, which also convert b and x "
                    "between the ABI and tiled layouts (4 more words per unknown)",
        },
        "stream_reference": ref,
        "setup_ms": setup_ms,
        "adjoint_step_ms": adj_ms,
        "autograd_step_ms": {"first": diff_first_ms, "reused": diff_ms,
                             "note": "helmholtz_solve(b, kh, kv, delta) forward + backward of "
                                     "g . x; the first call builds the operator, later ones "
                                     "reuse it with helmholtz_update"},
    }
    out["vcycle_in_solve"]["fp32"]["frac_of_stream"] = \
        out["vcycle_in_solve"]["fp32"]["GBps"] / stream_gbs
    x64_np = x64.cpu().numpy()
    x32_np = x32.cpu().numpy()
    xg = xref_gpu.cpu().numpy()
    err = lambda a, r: float(np.linalg.norm(a - r) / np.linalg.norm(r))  # noqa: E731
    out["fp32_mg"]["err_vs_gpu_fp64_1e-12"] = err(x32_np, xg)
    out["fp64_mg"]["err_vs_gpu_fp64_1e-12"] = err(x64_np, xg)
    del op32, op64, kh_d, kv_d, dl_d, xref_gpu
    torch.cuda.empty_cache()
    if not args.no_batch_leg and args.workload == "C192x70":
        out["batch4_C384x70"] = batch_leg(Operator, torch, dev)
    if not args.no_solver_comparison and args.workload == "C192x70":
        out["solver_comparison"] = solver_comparison(Operator, torch, dev)
    if not args.no_nine_cell and args.workload == "C192x70":
        out["nine_cell_C192x70"] = nine_cell_leg(Operator, torch, dev, _lib)
    if not args.no_weighted and args.workload == "C192x70":
        out["nonsymmetric_C192x70"] = weighted_leg(Operator, torch, dev)
    if baseline is not None:
        base, x_ref, x_6, big = finish_cpu_baseline(*baseline)
        out["cpu_baseline"] = base
        for key, xs in (("fp32_mg", x32_np), ("fp64_mg", x64_np)):
            out[key]["err_vs_oracle_1e-12"] = err(xs, x_ref)
            out[key]["err_vs_oracle_1e-6_iterate"] = err(xs, x_6)
        out["oracle_C192x70"] = {"iters_to_1e-6": big["iters"],
                                 "iters_to_1e-12": big["iters_to_1e-12"],
                                 "err_1e-6_iterate_vs_1e-12": err(x_6, x_ref)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
