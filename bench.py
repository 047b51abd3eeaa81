"""Benchmark of the batched Hermitian positive-definite inversion on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras]

Workload (one step): the MIMO-shaped batch -- 1,048,576 complex64 Hermitian
positive-definite matrices, half of order 8 and half of order 16,
A = B B^H + sigma I with sigma = 10^U(-2, 0) -- inverted by the Section IV
method in mixed precision (FP32 bulk, FP64 pivots, one Newton-Schulz step
with an FP64 residual).  Inputs are resident in HBM before timing; the step
is the two batched launches (one per order), taking three input/output sets
in turn.  `value` = inverses per second over the whole batch (elapsed time of
the K timed steps); the details also give the median, p10 and p90 of the
step and launch times.

The printed JSON line also carries
  roofline      for the kernel that dominates the step (mean per-launch
                duration from HIP events on its stream; algorithmic bytes per
                launch)
  cpu_baseline  the FP64 CPU oracle on a bounded sample: one pinned core (the
                value) and all usable cores (OpenMP over matrices), with the
                CPU model, core counts and compiler flags; it also compares the
                GPU's timed outputs for the sampled matrices with the oracle's
  details       per-order rates, the plain-FP64 path on the same matrices,
                errors of other workloads against FP64 LAPACK inverses
                (`*_vs_lapack`) or closed forms, the differentiation workload
                (forward + backward), the large single matrices and the other
                workloads.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12            # bytes/s, MI355X published HBM3E bandwidth
COUNT_PER_ORDER = 524288     # each half of the MIMO batch


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _pct(v, q):
    return float(np.percentile(np.asarray(v, dtype=np.float64), q))


def _time_loop(torch, fns, steps, warmup, stats=None):
    """Run `fns` (list of callables, each one kernel launch or graph replay) per
    step; return the mean step time (ms: elapsed over all steps / steps) and the
    mean per-launch duration of each fn (ms), all from HIP events on the
    current stream.  If `stats` is a dict it receives the median, p10 and p90
    of the step times and of each fn's launch durations."""
    for _ in range(warmup):
        for f in fns:
            f()
    torch.cuda.synchronize()
    per = [[_events(torch) for _ in range(steps)] for _ in fns]
    t0, t1 = _events(torch)
    t0.record()
    for s in range(steps):
        for i, f in enumerate(fns):
            per[i][s][0].record()
            f()
            per[i][s][1].record()
    t1.record()
    torch.cuda.synchronize()
    step_ms = t0.elapsed_time(t1) / steps
    durs = [[a.elapsed_time(b) for a, b in per[i]] for i in range(len(fns))]
    launch_ms = [float(np.mean(d)) for d in durs]
    if stats is not None:
        steps_ms = [per[0][s][0].elapsed_time(per[-1][s][1]) for s in range(steps)]
        stats["step_ms_median"] = _pct(steps_ms, 50)
        stats["step_ms_p10"] = _pct(steps_ms, 10)
        stats["step_ms_p90"] = _pct(steps_ms, 90)
        stats["launch_ms_median"] = [_pct(d, 50) for d in durs]
        stats["launch_ms_p10"] = [_pct(d, 10) for d in durs]
        stats["launch_ms_p90"] = [_pct(d, 90) for d in durs]
    return step_ms, launch_ms


def _ref_inv(a):
    """FP64 reference inverses from the CPU linear-algebra library (LU), for the
    accuracy figures reported next to the timings."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a).astype(
        np.complex128 if np.iscomplexobj(a) else np.float64))
    return torch.linalg.inv(t).numpy()


def _rel(x, ref):
    num = np.sqrt(np.sum(np.abs(x - ref) ** 2, axis=(-1, -2)))
    return num / np.sqrt(np.sum(np.abs(ref) ** 2, axis=(-1, -2)))


def _errors(x, a, idx):
    """max relative Frobenius error and max err/kappa over sampled matrices
    (reference: FP64 library inverse; kappa from FP64 library eigenvalues)."""
    import torch
    am = a[idx].astype(np.complex128)
    err = _rel(x[idx].astype(np.complex128), _ref_inv(am))
    ev = torch.linalg.eigvalsh(torch.from_numpy(am)).numpy()
    kap = ev[:, -1] / ev[:, 0]
    return float(err.max()), float((err / kap).max())


def _traffic(kernel_key, launches_bytes):
    """HBM traffic per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            tab = json.load(f)
        from paper_1111_4144_amd import build as B
        ent = tab.get(kernel_key)
        if not ent or ent.get("source_digest") != B.source_digest():
            return None
        return float(ent["fetch_bytes"] + ent["write_bytes"])
    except (OSError, ValueError, KeyError):
        return None


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(gpu_x=None, target_seconds=10.0):
    """The oracle (plain C, FP64) on the leading 65,536 matrices of each half of
    the MIMO batch, repeated until about target_seconds of CPU work: first on
    one core (the process pinned to one CPU with sched_setaffinity for the
    run), then the same routine with OpenMP over matrices on every CPU this
    process may use (at most 16, the host share of one GPU); matrices/s.
    If gpu_x = (x8, x16), the GPU's timed outputs for the same matrices, they
    are compared with the oracle's inverses (max relative Frobenius error)."""
    import oracle as O
    from paper_1111_4144_amd import inputs as G
    n_each = 65536
    a8 = G.mimo(8, n_each)
    a16 = G.mimo(16, n_each)
    cpus = sorted(os.sched_getaffinity(0))
    threads = min(len(cpus), 16)

    def run(fn, secs_target):
        done, t, outs = 0, time.perf_counter(), None
        while True:
            outs = (fn(a8), fn(a16))
            done += 2 * n_each
            secs = time.perf_counter() - t
            if secs >= secs_target:
                return done / secs, done // (2 * n_each), secs, outs

    os.sched_setaffinity(0, {cpus[0]})
    try:
        rate1, reps1, secs1, outs = run(O.inv_prop, target_seconds)
    finally:
        os.sched_setaffinity(0, set(cpus))
    rate_all, reps_all, secs_all, _ = run(lambda a: O.inv_prop_all_cores(a, threads),
                                          target_seconds / 2)
    res = {"value": rate1, "unit": "inverses/s", "cores": 1, "kind": "oracle",
           "sample": "first %d 8x8 + %d 16x16 matrices of the MIMO batch, inverted %d times "
                     "in complex128 by the oracle on one pinned core (%.1f s)"
                     % (n_each, n_each, reps1, secs1),
           "cpu_model": _cpu_model(), "nproc": os.cpu_count(), "affinity_cpus": len(cpus),
           "compiler": O.build_flags(),
           "all_cores": {"value": rate_all, "unit": "inverses/s", "cores": threads,
                         "sample": "same sample, OpenMP over matrices, %d repetitions (%.1f s)"
                                   % (reps_all, secs_all)}}
    if gpu_x is not None:
        errs = []
        for (xo, info), xg in zip(outs, gpu_x):
            assert not np.any(info)
            errs.append(float(_rel(xg[:n_each].astype(np.complex128), xo).max()))
        res["gpu_max_rel_err_vs_oracle_on_sample"] = max(errs)
    return res


FP32_MFMA_PEAK = 157.3e12
FP64_MFMA_PEAK = 78.6e12


def large_workloads(torch, api, G, dev, steps, tune=True):
    """Single large SPD matrices, A = Q diag(lambda) Q^T, lambda log-spaced over
    [1, 1e6], at N = 4096 and 8192: FP32 + FP64 pivots (factor + inverse, and
    with one Newton-Schulz step) and plain FP64.  Rates use the nominal N^3
    flops of factor + inverse (fraction of the FP32 or FP64 MFMA peak); with a
    refinement step the step adds 2 N^3 FP64 + N^3 FP32 flops, and its
    fraction is the sum of each part's time at its own peak over the measured
    time.  Errors: sampled entries against the closed form Q diag(1/lambda) Q^T
    (max abs error / ||X||_2), and the FP64 residual of 8 sampled columns
    against the stored input (max ||A x_j - e_j|| / (||A|| ||x_j||)).  The
    speedup of the mixed path (one refinement step) over plain FP64 is
    reported at each N with both errors."""
    out = {}
    rng = np.random.default_rng(1)
    for n in (4096, 8192):
        a, q, lam = G.large_spd(n, return_factors=True)
        idx = (rng.integers(0, n, 2048), rng.integers(0, n, 2048))
        ref = np.einsum("sk,sk->s", q[idx[0]] / lam[None, :], q[idx[1]])
        cols = rng.integers(0, n, 8)
        for dt, prec, ns_list, tag in [(torch.float32, "mixed", [0, 1], "fp32_mixed_%d" % n),
                                       (torch.float64, "plain", [0], "fp64_plain_%d" % n)]:
            A = torch.from_numpy(a).to(dev).to(dt)
            X = torch.empty_like(A)
            a_in = A.cpu().numpy().astype(np.float64)
            # configuration of the blocked path (diagonal kernel, inverse form,
            # split-K target) measured on this device for this order
            if tune:
                api.autotune(dt, precision=prec, orders=(n, n))
            out[tag + "_config"] = api.tuned_engine(dt, n, precision=prec)
            for ns in ns_list:
                st = {}
                step_ms, _ = _time_loop(
                    torch, [lambda: api.inverse(A, precision=prec, ns_steps=ns, out=X)], steps, 1,
                    stats=st)
                key = tag + ("_ns%d" % ns if prec == "mixed" else "")
                out[key + "_ms"] = step_ms
                out[key + "_ms_median"] = st["step_ms_median"]
                out[key + "_tflops_n3"] = n ** 3 / (step_ms / 1e3) / 1e12
                peak = FP32_MFMA_PEAK if dt == torch.float32 else FP64_MFMA_PEAK
                out[key + "_mfma_frac"] = n ** 3 / (step_ms / 1e3) / peak
                if ns > 0:
                    ideal = ns * (2 * n ** 3 / FP64_MFMA_PEAK + n ** 3 / FP32_MFMA_PEAK) + \
                        n ** 3 / FP32_MFMA_PEAK
                    out[key + "_mfma_frac_incl_refinement"] = ideal / (step_ms / 1e3)
                x = X.cpu().numpy()
                out[key + "_sampled_err_over_normX"] = float(
                    np.abs(x[idx].astype(np.float64) - ref).max() * lam.min())
                xc = x[:, cols].astype(np.float64)
                r = a_in @ xc
                r[cols, np.arange(cols.size)] -= 1.0
                out[key + "_fp64_residual"] = float(
                    (np.linalg.norm(r, axis=0) / (lam.max() * np.linalg.norm(xc, axis=0))).max())
                del x
            del A, X, a_in
            torch.cuda.empty_cache()
        out["speedup_mixed_ns1_vs_plain_fp64_%d" % n] = \
            out["fp64_plain_%d_ms" % n] / out["fp32_mixed_%d_ns1_ms" % n]
    return out


def varlen_workload(torch, api, G, dev, steps, tune=True):
    """262,144 real FP32 SPD matrices of orders U{2..64} in one packed buffer,
    one persistent launch (device bucketing prologue included), eager and as a
    replayed graph.  Bytes: A in + X out = 8 N^2 per matrix."""
    packed, sizes, offsets = G.varlen_spd(262144)
    P = torch.from_numpy(packed).to(dev)
    S = torch.from_numpy(sizes).to(dev)
    OF = torch.from_numpy(offsets).to(dev)
    XV = torch.empty_like(P)
    ws = torch.empty(api.varlen_workspace_bytes(P, S.shape[0]), dtype=torch.uint8, device=dev)
    # edge of the last size bucket, measured on this batch
    edge = api.autotune_varlen(P, S, OF, n_max=64, workspace=ws) if tune else 33

    def call():
        api.inverse_varlen(P, S, OF, n_max=64, out=XV, workspace=ws)

    e_ms, _ = _time_loop(torch, [call], steps, 2)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        call()
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            call()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g_ms, _ = _time_loop(torch, [g.replay], steps, 2)
    count = sizes.shape[0]
    nbytes = float(8 * np.sum(sizes.astype(np.int64) ** 2))
    x = XV.cpu().numpy()
    worst = 0.0
    for b in range(0, count, count // 256):
        n, o = int(sizes[b]), int(offsets[b])
        am = packed[o:o + n * n].reshape(n, n).astype(np.float64)
        xo = _ref_inv(am)
        xm = x[o:o + n * n].reshape(n, n)
        worst = max(worst, float(np.linalg.norm(xm - xo) / np.linalg.norm(xo)))
    del P, S, OF, XV, ws
    return {"varlen_eager_mat_per_s": count / (e_ms / 1e3),
            "varlen_graph_mat_per_s": count / (g_ms / 1e3),
            "varlen_graph_hbm_frac": nbytes / (g_ms / 1e3) / HBM_PEAK,
            "varlen_graph_ms": g_ms, "varlen_bucket_edge": edge,
            "varlen_sampled_max_rel_err_vs_lapack": worst}


def plain_small_workload(torch, api, G, dev, steps):
    """4096 complex128 4x4 matrices, plain FP64: launch time and error against
    the FP64 library inverse."""
    a = G.plain_fp64_4x4()
    A = torch.from_numpy(a).to(dev)
    X = torch.empty_like(A)
    ms, _ = _time_loop(torch, [lambda: api.inverse(A, out=X)], steps * 10, 5)
    xo = _ref_inv(a)
    x = X.cpu().numpy()
    err = np.sqrt(np.sum(np.abs(x - xo) ** 2, axis=(-1, -2))) / \
        np.sqrt(np.sum(np.abs(xo) ** 2, axis=(-1, -2)))
    return {"plain_c128_4x4_us_per_launch": ms * 1e3,
            "plain_c128_4x4_max_rel_err_vs_lapack": float(err.max())}


def solve_workload(torch, api, mats, steps):
    """Batched solves with one right-hand side per system from the factors of
    the MIMO batches (eqs. 5-7): time of the solve launch alone and of factor +
    solve.  Algorithmic bytes per system: the upper triangle of R, y and x."""
    out = {}
    g = torch.Generator(device=mats[0].device).manual_seed(3)
    for A in mats:
        count, n = A.shape[0], A.shape[-1]
        Rf = api.factor(A)
        Y = torch.randn((count, n), dtype=A.dtype, device=A.device, generator=g)
        X = torch.empty_like(Y)
        ms, (ls,) = _time_loop(torch, [lambda: api.solve_factored(Rf, Y, out=X)], steps, 2)
        fs_ms, _ = _time_loop(torch, [lambda: api.solve(A, Y)], max(2, steps // 2), 1)
        per_sys = (n * (n + 1) // 2 + 2 * n) * A.element_size()
        key = "solve_c64_%dx%d" % (n, n)
        out[key + "_per_s"] = count / (ls / 1e3)
        out[key + "_hbm_frac"] = count * per_sys / (ls / 1e3) / HBM_PEAK
        out[key + "_factor_plus_solve_per_s"] = count / (fs_ms / 1e3)
    return out


def nonherm_workload(torch, api, dev, steps):
    """General (non-Hermitian) complex64 8 x 8 inverses through D D^* (Section
    III.C), 524,288 per batch, mixed precision with one refinement step; the
    left-inverse residual max |X D - I| over the batch.  D = I + E with
    ||E||_2 about 0.35, so kappa(D) stays below about 2 and kappa(D D^*)
    below about 5 for every matrix of the batch."""
    n, count = 8, 1 << 19
    g = torch.Generator(device=dev).manual_seed(5)
    D = torch.randn((count, n, n), dtype=torch.complex64, device=dev, generator=g)
    D *= 0.125 / n ** 0.5
    D += torch.eye(n, dtype=torch.complex64, device=dev)
    state = {}

    def f():
        state["x"] = api.inverse_nonherm(D, precision="mixed", ns_steps=1)

    ms, _ = _time_loop(torch, [f], steps, 2)
    X = state["x"].to(torch.complex128)
    resid = (torch.matmul(X, D.to(torch.complex128)) - torch.eye(n, device=dev)).abs().amax()
    return {"nonherm_c64_8x8_inv_per_s": count / (ms / 1e3),
            "nonherm_c64_8x8_max_resid": float(resid)}


def q15_workload(torch, api, G, dev, steps):
    """Fixed-point inversion of the 8 x 8 half of the MIMO batch quantized to
    Q15 (524,288 matrices): rate, and the average relative Frobenius error
    against the FP64 inverse of the quantized matrices over a sample (the
    error measure of the paper's fixed-point comparison), for the proposed
    route and the two Section III methods in the same format; the share of
    sampled matrices where a Section III result equals the proposed one bit
    for bit."""
    n, count = 8, 1 << 19
    q, _ = G.quantize_q15(G.mimo(n, count))
    Q = torch.from_numpy(q).to(dev)
    idx = np.arange(0, count, count // 2048)
    at = (q[idx, ..., 0] + 1j * q[idx, ..., 1]).astype(np.complex128) / 2.0 ** 15
    ref = _ref_inv(at)
    out = {}
    first = None
    for variant, key in (("IV.A", "q15_c64_8x8"), ("III.A", "q15_IIIA_c64_8x8"),
                         ("III.B", "q15_IIIB_c64_8x8")):
        state = {}

        def f():
            state["r"] = api.inverse_q15(Q, variant=variant)

        ms, _ = _time_loop(torch, [f], steps, 2)
        x, xe = (t.cpu().numpy() for t in state["r"])
        xs = x[idx].astype(np.float64)
        got = (xs[..., 0] + 1j * xs[..., 1]) * np.ldexp(1.0, xe[idx])[:, None, None]
        err = _rel(got, ref)
        out[key + "_inv_per_s"] = count / (ms / 1e3)
        out[key + "_avg_norm_err_vs_lapack"] = float(err.mean())
        out[key + "_max_norm_err_vs_lapack"] = float(err.max())
        if first is None:
            first = (x[idx], xe[idx])
        else:
            same = np.all(x[idx] == first[0], axis=(1, 2, 3)) & (xe[idx] == first[1])
            out[key + "_share_equal_to_IVA"] = float(same.mean())
    return out


def compare_workload(torch, api, a8, A8, steps):
    """Side by side on the 8 x 8 half of the MIMO batch (524,288 complex64,
    plain FP32 arithmetic): the Section III.A and III.B comparison kernels,
    the Section IV route in the same framework (same factor code, LDS layout
    and arithmetic: the like-for-like reference, "IVsame"), and the proposed
    method's tuned plain-FP32 engine; rates and sampled errors against FP64
    library inverses.  The three framework kernels differ only by their route
    from R to X, so their time ratios read against the operation counts
    (N = 8: 252, 420 and 372 complex multiplies)."""
    out = {}
    idx = np.arange(0, a8.shape[0], a8.shape[0] // 1024)
    ref = _ref_inv(a8[idx])
    cases = [("IV", lambda: api.inverse(A8)),
             ("IVsame", lambda: api.inverse_compare(A8, variant="IV")),
             ("IIIA", lambda: api.inverse_compare(A8, variant="III.A")),
             ("IIIB", lambda: api.inverse_compare(A8, variant="III.B"))]
    for name, fn in cases:
        state = {}

        def f():
            state["x"] = fn()

        ms, _ = _time_loop(torch, [f], steps, 1)
        x = state["x"][idx].cpu().numpy().astype(np.complex128)
        out["compare_c64_8x8_%s_plain_inv_per_s" % name] = a8.shape[0] / (ms / 1e3)
        out["compare_c64_8x8_%s_plain_avg_rel_err_vs_lapack" % name] = float(_rel(x, ref).mean())
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-extras", action="store_true", help="skip the secondary workloads")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline")
    ap.add_argument("--no-large", action="store_true", help="skip the N=8192 / N=4096 workloads")
    ap.add_argument("--only", choices=["large", "varlen"], default=None,
                    help="run only one secondary workload and print its figures (for profiling)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the built-in engine choice (no autotuning launches, e.g. for "
                         "counter runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB three times (the reference "
                         "kernel for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs on a single MI355X and "
              "has no multi-GPU path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": src.numel() * 4, "launches": 3}))
        return

    from paper_1111_4144_amd import api, inputs as G

    if args.only:
        fn = {"large": lambda: large_workloads(torch, api, G, dev, max(2, args.steps // 4),
                                               not args.no_tune),
              "varlen": lambda: varlen_workload(torch, api, G, dev, max(3, args.steps // 2),
                                                not args.no_tune)}
        print(json.dumps({"only": args.only, "details": fn[args.only]()}), flush=True)
        return

    # engine choice per order, measured on this device before any timing
    tuned = {}
    for n in (8, 16):
        if not args.no_tune:
            api.autotune(torch.complex64, precision="mixed", ns_steps=1, orders=(n, n),
                         batch=COUNT_PER_ORDER)
        tuned[n] = api.tuned_engine(torch.complex64, n, precision="mixed")

    t_gen = time.perf_counter()
    a8 = G.mimo(8, COUNT_PER_ORDER)
    a16 = G.mimo(16, COUNT_PER_ORDER)
    gen_s = time.perf_counter() - t_gen
    A8 = torch.from_numpy(a8).to(dev)
    A16 = torch.from_numpy(a16).to(dev)
    X8 = torch.empty_like(A8)
    X16 = torch.empty_like(A16)
    # three input/output sets used in turn, so consecutive launches on one order
    # are 2.5 GB of other traffic apart (the 256 MB Infinity Cache cannot serve
    # the timed bytes); the first set's outputs are the ones checked below
    sets = [(A8, X8, A16, X16)] + [(A8.clone(), torch.empty_like(A8), A16.clone(),
                                    torch.empty_like(A16)) for _ in range(2)]
    torch.cuda.synchronize()
    turn = {"8": 0, "16": 0}

    def f8():
        a, x = sets[turn["8"] % 3][0:2]
        turn["8"] += 1
        api.inverse(a, precision="mixed", ns_steps=1, out=x)

    def f16():
        a, x = sets[turn["16"] % 3][2:4]
        turn["16"] += 1
        api.inverse(a, precision="mixed", ns_steps=1, out=x)

    st = {}
    step_ms, (ms8, ms16) = _time_loop(torch, [f8, f16], args.steps, args.warmup, stats=st)
    total = 2 * COUNT_PER_ORDER
    value = total / (step_ms / 1e3)
    # the checked outputs: one more launch on set 0 of each order
    api.inverse(A8, precision="mixed", ns_steps=1, out=X8)
    api.inverse(A16, precision="mixed", ns_steps=1, out=X16)
    torch.cuda.synchronize()
    del sets[1:]

    # roofline of the dominant kernel (algorithmic bytes: A in + X out, dense)
    dom = "16x16" if ms16 >= ms8 else "8x8"
    dom_ms = max(ms8, ms16)
    n_dom = 16 if dom == "16x16" else 8
    bytes_launch = COUNT_PER_ORDER * n_dom * n_dom * 8 * 2
    achieved = bytes_launch / (dom_ms / 1e3)
    kernel_key = "mimo_c64_%s_mixed_ns1" % dom
    roofline = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9,
                "unit": "GB/s", "frac": achieved / HBM_PEAK,
                "traffic": _traffic(kernel_key, bytes_launch),
                "kernel": kernel_key, "launch_ms": dom_ms,
                "bytes_per_launch": bytes_launch}

    details = {
        "rate_8x8_inv_per_s": COUNT_PER_ORDER / (ms8 / 1e3),
        "rate_16x16_inv_per_s": COUNT_PER_ORDER / (ms16 / 1e3),
        "hbm_frac_8x8": COUNT_PER_ORDER * 1024 / (ms8 / 1e3) / HBM_PEAK,
        "hbm_frac_16x16": COUNT_PER_ORDER * 4096 / (ms16 / 1e3) / HBM_PEAK,
        "launch_ms_8x8": ms8, "launch_ms_16x16": ms16,
        "launch_ms_median_8x8": st["launch_ms_median"][0],
        "launch_ms_p10_8x8": st["launch_ms_p10"][0], "launch_ms_p90_8x8": st["launch_ms_p90"][0],
        "launch_ms_median_16x16": st["launch_ms_median"][1],
        "launch_ms_p10_16x16": st["launch_ms_p10"][1],
        "launch_ms_p90_16x16": st["launch_ms_p90"][1],
        "step_ms_median": st["step_ms_median"], "step_ms_p10": st["step_ms_p10"],
        "step_ms_p90": st["step_ms_p90"], "timed_steps": args.steps, "buffer_sets": 3,
        "input_generation_s": gen_s,
        "tuned_engine_8x8": tuned[8], "tuned_engine_16x16": tuned[16],
    }

    # accuracy of the timed outputs against FP64 library inverses (sampled matrices)
    rng = np.random.default_rng(0)
    idx8 = rng.choice(COUNT_PER_ORDER, 1024, replace=False)
    idx16 = rng.choice(COUNT_PER_ORDER, 1024, replace=False)
    x8 = X8.cpu().numpy()
    x16 = X16.cpu().numpy()
    e8, r8 = _errors(x8, a8, idx8)
    e16, r16 = _errors(x16, a16, idx16)
    details["mixed_max_rel_err_vs_lapack"] = max(e8, e16)
    details["mixed_max_err_over_kappa_vs_lapack"] = max(r8, r16)
    gpu_sample = (x8[:65536].copy(), x16[:65536].copy())
    del x8, x16

    if not args.no_extras:
        # plain FP64 on the same matrices (complex128), the speedup baseline; its
        # engines are measured and chosen on this device like the mixed ones
        ptuned = {}
        for n in (8, 16):
            if not args.no_tune:
                api.autotune(torch.complex128, precision="plain", orders=(n, n),
                             batch=COUNT_PER_ORDER)
            ptuned[n] = api.tuned_engine(torch.complex128, n, precision="plain")
        B8 = A8.to(torch.complex128)
        B16 = A16.to(torch.complex128)
        Y8 = torch.empty_like(B8)
        Y16 = torch.empty_like(B16)
        p_ms, (p8, p16) = _time_loop(
            torch, [lambda: api.inverse(B8, out=Y8), lambda: api.inverse(B16, out=Y16)],
            max(3, args.steps // 2), 2)
        pe8, pr8 = _errors(Y8.cpu().numpy(), a8, idx8)
        pe16, pr16 = _errors(Y16.cpu().numpy(), a16, idx16)
        details["plain_fp64_inv_per_s"] = total / (p_ms / 1e3)
        details["plain_fp64_max_rel_err_vs_lapack"] = max(pe8, pe16)
        details["speedup_mixed_vs_plain_fp64"] = p_ms / step_ms
        # per order: c128 moves 2 x 16 bytes per entry (A in, X out)
        for n, ms_n in ((8, p8), (16, p16)):
            details["plain_c128_%dx%d_launch_ms" % (n, n)] = ms_n
            details["plain_c128_%dx%d_hbm_frac" % (n, n)] = \
                COUNT_PER_ORDER * n * n * 32 / (ms_n / 1e3) / HBM_PEAK
            details["plain_c128_tuned_engine_%dx%d" % (n, n)] = ptuned[n]
        del B8, B16, Y8, Y16
        # mixed precision without refinement and plain FP32, for context
        z_ms, _ = _time_loop(torch, [lambda: api.inverse(A8, precision="mixed", ns_steps=0, out=X8),
                                     lambda: api.inverse(A16, precision="mixed", ns_steps=0, out=X16)],
                             max(3, args.steps // 2), 2)
        details["mixed_ns0_inv_per_s"] = total / (z_ms / 1e3)
        # differentiation workload: 65,536 complex64 16x16, forward + backward
        ag, gg = G.grad_16()
        AG = torch.from_numpy(ag).to(dev)
        GG = torch.from_numpy(gg).to(dev)
        XG = torch.empty_like(AG)
        state = {}

        def fwd():
            api.inverse(AG, precision="mixed", ns_steps=1, out=XG)

        def bwd():
            state["ga"] = api.inverse_backward(XG, GG)

        g_ms, (gf, gb) = _time_loop(torch, [fwd, bwd], max(3, args.steps // 2), 2)
        details["grad16_fwd_bwd_inv_per_s"] = ag.shape[0] / (g_ms / 1e3)
        details["grad16_bwd_hbm_frac"] = ag.shape[0] * 6144 / (gb / 1e3) / HBM_PEAK
        ga = state["ga"].cpu().numpy()
        sub = np.arange(0, ag.shape[0], 64)
        xo = _ref_inv(ag[sub])
        gh = 0.5 * (gg[sub] + np.conj(np.swapaxes(gg[sub], -1, -2)))
        want = -(xo @ gh @ xo)
        gerr = np.sqrt(np.sum(np.abs(ga[sub] - want) ** 2, axis=(-1, -2))) / \
            np.sqrt(np.sum(np.abs(want) ** 2, axis=(-1, -2)))
        details["grad16_max_rel_err_vs_lapack"] = float(gerr.max())
        del AG, GG, XG

    if not args.no_extras:
        details.update(solve_workload(torch, api, [A8, A16], max(3, args.steps // 2)))
        details.update(nonherm_workload(torch, api, dev, max(3, args.steps // 2)))
        details.update(q15_workload(torch, api, G, dev, max(3, args.steps // 2)))
        details.update(compare_workload(torch, api, a8, A8, max(3, args.steps // 4)))
    if not args.no_extras and not args.no_large:
        details.update(large_workloads(torch, api, G, dev, max(2, args.steps // 4),
                                       not args.no_tune))
    if not args.no_extras:
        details.update(varlen_workload(torch, api, G, dev, max(3, args.steps // 2),
                                       not args.no_tune))
        details.update(plain_small_workload(torch, api, G, dev, max(3, args.steps // 2)))

    line = {
        "metric": "inverses/s (8x8 c64 batch), TFLOP/s N=8192, fwd+bwd vs plain @ stated err",
        "value": value, "unit": "inverses/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": step_ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64 (FP32 + FP64 pivots/residual)",
        "data": "synthetic (seeded A = B B^H + sigma I)",
        "config": {"workload": "MIMO batch: 524,288 8x8 + 524,288 16x16 complex64 HPD, "
                               "mixed precision, 1 Newton-Schulz step", "global_batch": total,
                   "orders": [8, 16], "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": None if args.no_cpu else cpu_baseline(gpu_sample),
        "details": details,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
