"""Throughput of the filtered RK4 step on one MI355X.

Workload (default): a perturbed Kerr-Schild black hole (M = 1) on one shell
r in [1.8, 11.8] with 33 x 32 x 64 points, 50 GHG fields, Yn filter n_f = 4
after every step, Courant factor 4, FP64.  One step = 4 right-hand-side
evaluations (3 derivative contractions per field, pointwise GHG rhs with the
outer boundary operator and the RK stage update) + 1 tensor filter.

Prints ONE JSON line: field-points/s = n_fields * N_r * N_theta * N_phi /
time per step, the dominant kernel's roofline figures (its own launches timed
with HIP events on the stream it runs on, during the timed steps), and the
CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DESCRIPTIONS = {
    "ks33": "perturbed Kerr-Schild M=1, 1 shell 33x32x64 r[1.8,11.8], 50 GHG fields, Yn n_f=4, lambda=4, FP64",
    "ks49": "perturbed Kerr-Schild M=1, 1 shell 49x48x96 r[1.8,11.8], 50 GHG fields, Yn n_f=4, lambda=4, FP64",
}


def log(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print("[bench %7.1fs] %s" % (time.perf_counter() - T_START, msg), file=sys.stderr, flush=True)


T_START = time.perf_counter()


def algorithmic_bytes(cls, n_r, n_th, n_ph, n_v, K):
    """HBM bytes a kernel class must move per launch (FP64), per field-point
    times the field-points of one shell."""
    fp = n_v * n_r * n_th * n_ph
    npts = n_r * n_th * n_ph
    per_fp = {
        "d_r": 16.0, "d_theta": 16.0, "d_phi": 16.0,
        # stages read u (8), du (24), plus base/acc traffic: 48, 64, 64, 48 B -> mean 56
        "rhs_stage": 56.0,
        "filter_decompose": 16.0, "filter_recompose": 16.0,
        "filter_phi_analysis": 8.0 + 8.0 * K / n_ph,
        "filter_theta": 16.0 * K / n_ph,
        "filter_phi_synthesis": 8.0 + 8.0 * K / n_ph,
    }[cls]
    extra = 16 * 8 * npts if cls == "rhs_stage" else 0   # static gauge H_a, d_i H_b
    return per_fp * fp + extra


KERNEL_SOURCES = {"d_r": "tile_dr.h", "d_theta": "derivs.hip", "d_phi": "derivs.hip", "rhs_stage": "rhs.hip",
                  "filter_decompose": "filter.hip", "filter_recompose": "filter.hip", "filter_theta": "filter.hip",
                  "filter_phi_analysis": "derivs.hip", "filter_phi_synthesis": "derivs.hip"}


def profiled_traffic(workload, cls):
    """HBM bytes per launch of a kernel class from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, each scaled by the reading of a copy
    kernel of known size), or None when there is none or the kernel's source
    file has changed since the counters were taken (sha256 recorded there)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_%s.md" % workload)
    if not os.path.exists(path):
        return None
    src = KERNEL_SOURCES[cls]
    want, val = None, None
    for line in open(path):
        if line.startswith("source-sha256 %s " % src):
            want = line.split()[2]
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 6 and cells[0] == cls:
            try:
                val = float(cells[5])
            except ValueError:
                val = None
    if want is None or val is None:
        return None
    have = hashlib.sha256(open(os.path.join(ROOT, "paper_1104_3408_amd", "csrc", src), "rb").read()).hexdigest()
    return val if have == want else None


def run_variant(shells, n_v, precision, steps, warmup, seed0):
    """Throughput of one workload: seeded perturbed Kerr-Schild data on every
    shell (seed0 + shell index), filtered RK4 steps with the step graph."""
    import numpy as np
    import torch
    from paper_1104_3408_amd import shellspec as ss
    from paper_1104_3408_amd import inputs
    g = ss.ShellGrid(shells, n_fields=n_v, filter="Yn", n_f=4, courant=4.0, precision=precision)
    log("grid of %d shells created (precision %d)" % (len(shells), precision))
    g10, extra = [], []
    for k in range(len(shells)):
        r, th, ph = g.coords(k)
        g10.append(inputs.perturbed_kerr_schild(seed0 + k, r, th, ph).ravel())
        if n_v == 58:
            dH, Q = inputs.gauge_perturbation(seed0 + 1000 + k, r, th, ph)
            extra.append(np.concatenate([dH, Q]).ravel())
    u = torch.zeros(g.state_size, dtype=torch.float64, device="cuda")
    ex = torch.from_numpy(np.concatenate(extra)).cuda() if extra else None
    g.kerr_schild_data(torch.from_numpy(np.concatenate(g10)).cuda(), u, extra8=ex)
    del g10, extra, ex
    norms = torch.zeros(4 * len(shells), dtype=torch.float64, device="cuda")

    def constraint_norms():
        """max over shells of (max |C_a|, rms C_a, max |C_iab|, rms C_iab)"""
        g.ghg_constraints(u, norms)
        return [float(x) for x in norms.view(-1, 4).max(dim=0).values.cpu()]
    c0 = constraint_norms()
    g.rk_step(u, warmup)
    torch.cuda.synchronize()
    log("initial data and %d warmup steps done" % warmup)
    t0 = time.perf_counter()
    g.rk_step(u, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log("%d timed steps: %.3f ms/step" % (steps, 1e3 * (t1 - t0) / steps))
    fp = sum(n_v * a * b * c for (a, b, c, _, _) in shells)
    res = {"field_points": fp, "ms_per_step": 1e3 * (t1 - t0) / steps, "value": fp * steps / (t1 - t0),
           "steps": steps, "state_finite": bool(torch.isfinite(u).all().item()),
           "constraints_max_abs_rms_Ca_Ciab": {"initial": c0, "after_%d_steps" % (warmup + steps): constraint_norms()}}
    return res, u, g


def fft_vs_matmul(reps=20):
    """d_phi by the library's Fourier-matrix contraction against an FFT route
    (torch.fft on ROCm: real FFT along phi, multiply by i m with the Nyquist
    mode dropped, inverse FFT) on the same [field][phi][theta][r] layout, for
    33 x N_theta x 2 N_theta shells with 50 fields.  Microseconds per call,
    and the largest difference between the two results relative to max|d_phi u|."""
    import torch
    from paper_1104_3408_amd import shellspec as ss
    rows = []
    for n_th in (4, 8, 16, 24, 32, 48, 64):
        n_ph, n_r = 2 * n_th, 33
        g = ss.ShellGrid([(n_r, n_th, n_ph, 1.8, 11.8)])
        gen = torch.Generator(device="cuda").manual_seed(n_th)
        u = torch.randn(g.state_size, dtype=torch.float64, device="cuda", generator=gen)
        du = torch.empty(3 * g.state_size, dtype=torch.float64, device="cuda")
        g.spec_derivs(u, du)
        g.enable_timing(True)
        for _ in range(reps):
            g.spec_derivs(u, du)
        torch.cuda.synchronize()
        ms, cnt = g.kernel_times()
        g.enable_timing(False)
        k = ss.KERNEL_CLASSES.index("d_phi")
        mm_us = 1e3 * ms[k] / max(cnt[k], 1)
        v = u.view(50, n_ph, n_th * n_r)
        mult = 1j * torch.arange(n_ph // 2 + 1, device="cuda", dtype=torch.float64)
        mult[-1] = 0.0                                     # Nyquist mode carries no derivative
        mult = mult.view(1, -1, 1)

        def fft_dphi():
            return torch.fft.irfft(torch.fft.rfft(v, dim=1) * mult, n=n_ph, dim=1)

        out = fft_dphi()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            out = fft_dphi()
        e1.record()
        torch.cuda.synchronize()
        fft_us = 1e3 * e0.elapsed_time(e1) / reps
        ref = du[2 * g.state_size:].view(50, n_ph, n_th * n_r)
        diff = float((out - ref).abs().max() / ref.abs().max())
        rows.append({"n_phi": n_ph, "matmul_us": round(mm_us, 2), "fft_us": round(fft_us, 2),
                     "fft_over_matmul": round(fft_us / mm_us, 2), "max_rel_diff": diff})
        del g, u, du, out
    return rows


def cpu_baseline(shell, g10, dt, gpu_state_after_one_step):
    """Oracle (numpy FP64) on one filtered RK4 step of the same workload."""
    import numpy as np
    from oracle.grid import Shell
    from oracle import initial_data as oid
    from oracle.evolve import Evolution
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = 1
    n_r, n_th, n_ph, a, b = shell
    sh = Shell(n_r, n_th, n_ph, a, b)
    u0 = oid.first_order_data(g10, sh)
    H, dH = oid.static_gauge(u0, sh)
    ev = Evolution(sh, 50, H, dH, "Yn", 4)
    t0 = time.perf_counter()
    ref = ev.rk4_step(u0, dt)
    t1 = time.perf_counter()
    fp = 50 * sh.npts
    got = gpu_state_after_one_step.reshape(ref.shape)
    err = np.abs(got - ref)
    scale = np.abs(ref).max()
    rms = float(np.sqrt(np.mean(err ** 2)) / np.sqrt(np.mean(ref ** 2)))
    return ({"value": fp / (t1 - t0), "unit": "field-points/s", "cores": int(threads), "kind": "oracle",
             "sample": "1 filtered RK4 step of the same shell (%dx%dx%d, 50 fields), %.1f s" % (n_r, n_th, n_ph,
                                                                                               t1 - t0)},
            {"max_rel": float(err.max() / scale), "rms_rel": rms, "after_steps": 1})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="ks33", choices=sorted(DESCRIPTIONS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true", help="skip the per-kernel HIP events")
    ap.add_argument("--no-variants", action="store_true", help="skip the mixed-precision and batched workloads")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="run one device copy of this many MiB (a known-size kernel for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (shells are independent and would be "
              "assigned to GPUs whole, with no exchange during a step); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1104_3408_amd import shellspec as ss
    from paper_1104_3408_amd import inputs

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    shells, n_v = inputs.workload_shells(args.workload)
    desc = DESCRIPTIONS[args.workload]
    seed0 = inputs.WORKLOAD_SEED[args.workload]
    g = ss.ShellGrid(shells, n_fields=n_v, filter="Yn", n_f=4, courant=4.0)
    log("grid created")
    g10 = []
    for k in range(len(shells)):
        r, th, ph = g.coords(k)
        g10.append(inputs.perturbed_kerr_schild(seed0 + k, r, th, ph).ravel())
    g10 = np.concatenate(g10)
    u = torch.zeros(g.state_size, dtype=torch.float64, device="cuda")
    g.kerr_schild_data(torch.from_numpy(g10).cuda(), u)
    stream = torch.cuda.current_stream()

    # one step for the error statement, from the same initial data
    u1 = u.clone()
    g.rk_step(u1, 1)
    torch.cuda.synchronize()
    u1_host = u1.cpu().numpy()
    del u1

    g.rk_step(u, args.warmup)
    torch.cuda.synchronize()
    # timed region: K filtered steps, one captured step graph replayed per step
    t0 = time.perf_counter()
    g.rk_step(u, args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    fp = sum(n_v * a * b * c for (a, b, c, _, _) in shells)
    ms_per_step = 1e3 * elapsed / args.steps
    value = fp * args.steps / elapsed
    finite = bool(torch.isfinite(u).all().item())
    log("timed region: %d steps, %.4f ms/step" % (args.steps, ms_per_step))

    out = {"metric": "field-points/s per filtered RK4 step", "value": value, "unit": "field-points/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic", "config": {"workload": desc, "shells": [list(s) for s in shells],
                                          "n_fields": n_v, "filter": "Yn", "n_f": 4, "courant": 4.0,
                                          "field_points": fp, "state_finite": finite}}
    if not args.no_timing:
        # second timed pass of K steps with HIP events around every launch, on the
        # stream the kernels run on (the eager launch path; events sit between launches)
        g.enable_timing(True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        g.rk_step(u, args.steps)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        ms, cnt = g.kernel_times()
        g.enable_timing(False)
        kern = {c: {"total_ms": ms[i], "launches": cnt[i], "avg_us": 1e3 * ms[i] / max(cnt[i], 1)}
                for i, c in enumerate(ss.KERNEL_CLASSES)}
        dom = max(kern, key=lambda c: kern[c]["total_ms"])
        byts = sum(algorithmic_bytes(dom, *s[:3], n_v, 2 * (s[1] - 1 - 4) + 1) for s in shells)
        avg_s = kern[dom]["avg_us"] * 1e-6
        ach = byts / avg_s / 1e9
        out["roofline"] = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": ach / HBM_PEAK_GBS, "traffic": profiled_traffic(args.workload, dom),
                           "bytes_per_launch": byts, "avg_launch_us": kern[dom]["avg_us"]}
        out["kernels"] = kern
        out["timing_pass_ms_per_step"] = 1e3 * (t3 - t2) / args.steps
        tot = sum(k["total_ms"] for k in kern.values())
        out["kernel_time_share"] = {c: kern[c]["total_ms"] / tot for c in kern}
        log("timing pass done, dominant kernel %s %.2f us" % (dom, kern[dom]["avg_us"]))
    if args.copy_probe_mb:
        src = torch.empty(args.copy_probe_mb * (1 << 20) // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes_each_way"] = src.numel() * 8
        del src, dst
    if not args.no_variants:
        var = {}
        # same shell, angular derivatives in FP32; error vs the FP64 GPU state
        # (which matches the oracle to 1e-12) after the same number of steps
        res, um, gm = run_variant(shells, n_v, ss.SG_PREC_FP32, args.steps, args.warmup, seed0)
        res64, uref, gr = run_variant(shells, n_v, ss.SG_PREC_FP64, args.steps, args.warmup, seed0)
        d = (um - uref).abs().max().item() / uref.abs().max().item()
        res["max_rel_diff_vs_fp64_gpu"] = d
        res["speedup_vs_fp64"] = res["value"] / res64["value"]
        var["mixed_fp32_angular"] = res
        del um, gm
        # angular contractions on the matrix cores from two-part bfloat16
        # operands (the filter as in the FP32 mode)
        rb, ub, gb = run_variant(shells, n_v, ss.SG_PREC_BF16X3, args.steps, args.warmup, seed0)
        rb["max_rel_diff_vs_fp64_gpu"] = (ub - uref).abs().max().item() / uref.abs().max().item()
        rb["speedup_vs_fp64"] = rb["value"] / res64["value"]
        var["mixed_bf16x3_angular"] = rb
        del ub, gb, uref, gr
        for name, steps in (("batch64", 20), ("large8", 10)):
            bshells, bnv = inputs.workload_shells(name)
            bseed = inputs.WORKLOAD_SEED[name]
            r64, u64, g64 = run_variant(bshells, bnv, ss.SG_PREC_FP64, steps, 2, bseed)
            u64h = u64.clone()
            del u64, g64
            torch.cuda.empty_cache()
            r32, u32, g32 = run_variant(bshells, bnv, ss.SG_PREC_FP32, steps, 2, bseed)
            r32["max_rel_diff_vs_fp64_gpu"] = (u32 - u64h).abs().max().item() / u64h.abs().max().item()
            r32["speedup_vs_fp64"] = r32["value"] / r64["value"]
            del u32, g32
            torch.cuda.empty_cache()
            rb, ub, gb = run_variant(bshells, bnv, ss.SG_PREC_BF16X3, steps, 2, bseed)
            rb["max_rel_diff_vs_fp64_gpu"] = (ub - u64h).abs().max().item() / u64h.abs().max().item()
            rb["speedup_vs_fp64"] = rb["value"] / r64["value"]
            var[name] = {"shells": len(bshells), "n_fields": bnv, "fp64": r64, "mixed_fp32_angular": r32,
                         "mixed_bf16x3_angular": rb}
            del ub, gb, u64h
            torch.cuda.empty_cache()
        var["fft_vs_matmul_dphi"] = fft_vs_matmul()
        log("FFT comparison done")
        out["variants"] = var
    if not args.no_cpu_baseline and len(shells) == 1:
        log("oracle step on the host")
        base, err = cpu_baseline(shells[0], g10.reshape((10,) + (shells[0][2], shells[0][1], shells[0][0])),
                                 g.info(0)[2], u1_host)
        out["cpu_baseline"] = base
        out["error_vs_oracle"] = err
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
