"""Benchmark of the batched Hermitian positive-definite inversion on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras]

Workload (one step): the MIMO-shaped batch -- 1,048,576 complex64 Hermitian
positive-definite matrices, half of order 8 and half of order 16,
A = B B^H + sigma I with sigma = 10^U(-2, 0) -- inverted by the Section IV
method in mixed precision (FP32 bulk, FP64 pivots, one Newton-Schulz step
with an FP64 residual).  Inputs are resident in HBM before timing; the step
is the two batched launches (one per order).  `value` = inverses per second
over the whole batch.

The printed JSON line also carries
  roofline      for the kernel that dominates the step (per-launch duration
                from HIP events on its stream; algorithmic bytes per launch)
  cpu_baseline  the FP64 CPU oracle, single-threaded, on a bounded sample
  details       per-order rates, the plain-FP64 path on the same matrices, the
                measured errors against FP64 library inverses (the oracle is
                used by the CPU baseline only), the differentiation workload
                (forward + backward), and the other workloads.
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


def _time_loop(torch, fns, steps, warmup):
    """Run `fns` (list of callables, each one kernel launch) per step; return the
    mean step time (ms) and the mean per-launch duration of each fn (ms), all
    measured with HIP events on the current stream."""
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
    launch_ms = [float(np.mean([a.elapsed_time(b) for a, b in per[i]])) for i in range(len(fns))]
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


def cpu_baseline(target_seconds=10.0):
    """The oracle (plain C, FP64, one thread) on the leading 65,536 matrices of each
    half of the MIMO batch, repeated until about target_seconds of CPU work;
    matrices/s."""
    import oracle as O
    from paper_1111_4144_amd import inputs as G
    n_each = 65536
    a8 = G.mimo(8, n_each)
    a16 = G.mimo(16, n_each)
    done = 0
    t = time.perf_counter()
    while True:
        O.inv_prop(a8)
        O.inv_prop(a16)
        done += 2 * n_each
        secs = time.perf_counter() - t
        if secs >= target_seconds:
            break
    return {"value": done / secs, "unit": "inverses/s", "cores": 1, "kind": "oracle",
            "sample": "first %d 8x8 + %d 16x16 matrices of the MIMO batch, inverted %d times "
                      "in complex128 by the single-threaded oracle (%.1f s)"
                      % (n_each, n_each, done // (2 * n_each), secs)}


FP32_MFMA_PEAK = 157.3e12
FP64_MFMA_PEAK = 78.6e12


def large_workloads(torch, api, G, dev, steps):
    """Single large SPD matrices, A = Q diag(lambda) Q^T, lambda log-spaced over
    [1, 1e6]: FP32 + FP64 pivots at N=8192 (factor + inverse, then with one
    Newton-Schulz step) and plain FP64 at N=4096.  Rates use the nominal N^3
    flops of factor + inverse; a refinement step adds 2 N^3 (FP64) + N^3 (FP32)."""
    out = {}
    rng = np.random.default_rng(1)
    for n, dt, prec, tag in [(8192, torch.float32, "mixed", "fp32_mixed_8192"),
                             (4096, torch.float64, "plain", "fp64_plain_4096")]:
        a, q, lam = G.large_spd(n, return_factors=True)
        A = torch.from_numpy(a).to(dev).to(dt)
        X = torch.empty_like(A)
        ns_list = [0, 1] if prec == "mixed" else [0]
        for ns in ns_list:
            step_ms, _ = _time_loop(
                torch, [lambda: api.inverse(A, precision=prec, ns_steps=ns, out=X)], steps, 1)
            key = tag + ("_ns%d" % ns if prec == "mixed" else "")
            out[key + "_ms"] = step_ms
            out[key + "_tflops_n3"] = n ** 3 / (step_ms / 1e3) / 1e12
            if ns == 0:
                peak = FP32_MFMA_PEAK if dt == torch.float32 else FP64_MFMA_PEAK
                out[key + "_mfma_frac"] = n ** 3 / (step_ms / 1e3) / peak
            # sampled entries against the closed form Q diag(1/lambda) Q^T
            idx = (rng.integers(0, n, 2048), rng.integers(0, n, 2048))
            xs = X.cpu().numpy().astype(np.float64)[idx]
            ref = np.einsum("sk,sk->s", q[idx[0]] / lam[None, :], q[idx[1]])
            out[key + "_sampled_err_over_normX"] = float(np.abs(xs - ref).max() * lam.min())
        del A, X
        torch.cuda.empty_cache()
    return out


def varlen_workload(torch, api, G, dev, steps):
    """262,144 real FP32 SPD matrices of orders U{2..64} in one packed buffer,
    one persistent launch (device bucketing prologue included), eager and as a
    replayed graph.  Bytes: A in + X out = 8 N^2 per matrix."""
    packed, sizes, offsets = G.varlen_spd(262144)
    P = torch.from_numpy(packed).to(dev)
    S = torch.from_numpy(sizes).to(dev)
    OF = torch.from_numpy(offsets).to(dev)
    XV = torch.empty_like(P)
    ws = torch.empty(api.varlen_workspace_bytes(P, S.shape[0]), dtype=torch.uint8, device=dev)

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
            "varlen_graph_ms": g_ms,
            "varlen_sampled_max_rel_err": worst}


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
            "plain_c128_4x4_max_rel_err": float(err.max())}


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
    error measure of the paper's fixed-point comparison)."""
    n, count = 8, 1 << 19
    q, _ = G.quantize_q15(G.mimo(n, count))
    Q = torch.from_numpy(q).to(dev)
    state = {}

    def f():
        state["r"] = api.inverse_q15(Q)

    ms, _ = _time_loop(torch, [f], steps, 2)
    x, xe = (t.cpu().numpy() for t in state["r"])
    idx = np.arange(0, count, count // 2048)
    at = (q[idx, ..., 0] + 1j * q[idx, ..., 1]).astype(np.complex128) / 2.0 ** 15
    ref = _ref_inv(at)
    xs = x[idx].astype(np.float64)
    got = (xs[..., 0] + 1j * xs[..., 1]) * np.ldexp(1.0, xe[idx])[:, None, None]
    err = _rel(got, ref)
    return {"q15_c64_8x8_inv_per_s": count / (ms / 1e3),
            "q15_c64_8x8_avg_norm_err": float(err.mean()),
            "q15_c64_8x8_max_norm_err": float(err.max())}


def compare_workload(torch, api, a8, A8, steps):
    """Side by side on the 8 x 8 half of the MIMO batch (524,288 complex64,
    plain FP32 arithmetic): the Section III.A and III.B comparison kernels and
    the proposed method's plain-FP32 engine; rates and sampled errors against
    FP64 library inverses (the comparison kernels are straightforward one-lane
    implementations, so their rates are context, not tuned baselines)."""
    out = {}
    idx = np.arange(0, a8.shape[0], a8.shape[0] // 1024)
    ref = _ref_inv(a8[idx])
    cases = [("IV", lambda: api.inverse(A8)),
             ("IIIA", lambda: api.inverse_compare(A8, variant="III.A")),
             ("IIIB", lambda: api.inverse_compare(A8, variant="III.B"))]
    for name, fn in cases:
        state = {}

        def f():
            state["x"] = fn()

        ms, _ = _time_loop(torch, [f], steps, 1)
        x = state["x"][idx].cpu().numpy().astype(np.complex128)
        out["compare_c64_8x8_%s_plain_inv_per_s" % name] = a8.shape[0] / (ms / 1e3)
        out["compare_c64_8x8_%s_plain_avg_rel_err" % name] = float(_rel(x, ref).mean())
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
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
        print("bench.py measures one GPU only: this build runs on a single MI355X and "
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
        fn = {"large": lambda: large_workloads(torch, api, G, dev, max(2, args.steps // 4)),
              "varlen": lambda: varlen_workload(torch, api, G, dev, max(3, args.steps // 2))}
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
    torch.cuda.synchronize()

    def f8():
        api.inverse(A8, precision="mixed", ns_steps=1, out=X8)

    def f16():
        api.inverse(A16, precision="mixed", ns_steps=1, out=X16)

    step_ms, (ms8, ms16) = _time_loop(torch, [f8, f16], args.steps, args.warmup)
    total = 2 * COUNT_PER_ORDER
    value = total / (step_ms / 1e3)

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
    details["mixed_max_rel_err"] = max(e8, e16)
    details["mixed_max_err_over_kappa"] = max(r8, r16)
    del x8, x16

    if not args.no_extras:
        # plain FP64 on the same matrices (complex128), the speedup baseline
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
        details["plain_fp64_max_rel_err"] = max(pe8, pe16)
        details["speedup_mixed_vs_plain_fp64"] = p_ms / step_ms
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
        details["grad16_max_rel_err"] = float(gerr.max())
        del AG, GG, XG

    if not args.no_extras:
        details.update(solve_workload(torch, api, [A8, A16], max(3, args.steps // 2)))
        details.update(nonherm_workload(torch, api, dev, max(3, args.steps // 2)))
        details.update(q15_workload(torch, api, G, dev, max(3, args.steps // 2)))
        details.update(compare_workload(torch, api, a8, A8, max(3, args.steps // 4)))
    if not args.no_extras and not args.no_large:
        details.update(large_workloads(torch, api, G, dev, max(2, args.steps // 4)))
    if not args.no_extras:
        details.update(varlen_workload(torch, api, G, dev, max(3, args.steps // 2)))
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
        "cpu_baseline": None if args.no_cpu else cpu_baseline(),
        "details": details,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
