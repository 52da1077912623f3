"""Throughput of the filtered RK4 step on one MI355X.

Workload (default, batch64): 64 independent shells of four sizes, 16 each of
17x16x32, 25x24x48, 33x32x64 and 49x48x96 (N_r x N_theta x N_phi, r in
[1.8, 11.8]), each a Kerr-Schild black hole (M = 1) with its own seeded smooth
perturbation of amplitude 1e-6; 50 GHG fields, Yn filter n_f = 4 after every
step, Courant factor 4, per-shell time step, FP64, one captured step graph
replayed per step (264.7M field-points, a 2.1 GB state: HBM-resident).  One
step = 4 right-hand-side evaluations (3 derivative contractions per field,
pointwise GHG rhs with the outer boundary operator and the RK stage update)
+ 1 tensor filter.

Prints ONE JSON line: field-points/s = sum over shells of n_fields N_r
N_theta N_phi / time per step; the dominant kernel's roofline figures (its own
launches timed with HIP events on the stream it runs on, in a second pass of
the same steps) and every kernel class's fraction of the HBM peak; the
mixed-precision forms of the same workload (FP32 and BF16x3 angular
contractions) with their speed-up; the error of every form against the CPU
oracle (one shell per size class after one step, max and RMS); the other
configurations (one 33x32x64 shell, one 49x48x96 shell in three precisions,
8 shells of 65x64x128 with 58 fields) with their errors against the stored
oracle evolutions after 1, 10 and 100 steps; four nested shells coupled at
their shared spheres against the same shells uncoupled, and the Y and Yg
filters against Yn on the 33x32x64 shell; and the oracle timed on the
host on a bounded sample of the workload, on all cores and on one core; and
the HBM bandwidth a plain device copy attains on this machine, beside the 8 TB/s
specification the roofline fractions use.
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
    "batch64": "64 perturbed Kerr-Schild shells, 16 each of 17x16x32, 25x24x48, 33x32x64, 49x48x96 r[1.8,11.8], "
               "50 GHG fields, Yn n_f=4, lambda=4, FP64",
    "large8": "8 perturbed Kerr-Schild shells 65x64x128 r[1.8,21.8], 58 fields (GHG + gauge source), Yn n_f=4, "
              "lambda=4, FP64",
    "ks33": "perturbed Kerr-Schild M=1, 1 shell 33x32x64 r[1.8,11.8], 50 GHG fields, Yn n_f=4, lambda=4, FP64",
    "ks49": "perturbed Kerr-Schild M=1, 1 shell 49x48x96 r[1.8,11.8], 50 GHG fields, Yn n_f=4, lambda=4, FP64",
}
PREC_NAMES = {0: "fp64", 1: "fp32_angular", 2: "bf16x3_angular"}


def log(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print("[bench %7.1fs] %s" % (time.perf_counter() - T_START, msg), file=sys.stderr, flush=True)


T_START = time.perf_counter()


def k_keep(n_th, n_f=4):
    """Real phi modes the Yn filter keeps: 2 (N_theta - 1 - n_f) + 1."""
    return 2 * (n_th - 1 - n_f) + 1


def bytes_per_launch(cls, shell, n_v, count=1):
    """Algorithmic HBM bytes of one FP64 launch of a kernel class on a run of
    `count` identical shells: bytes per field-point times the field-points
    (plus, for the rhs, 128 B per grid point of static gauge H_a, d_i H_b
    with 50 fields)."""
    n_r, n_th, n_ph = shell[:3]
    fp = n_v * n_r * n_th * n_ph * count
    npts = n_r * n_th * n_ph * count
    K = k_keep(n_th)
    per_fp = {
        "d_r": 16.0, "d_theta": 16.0, "d_phi": 16.0,
        "derivs_fused": 32.0,   # u read once, three derivatives written
        # stages read u (8), du (24), plus base/acc traffic: 48, 64, 64, 48 B -> mean 56
        "rhs_stage": 56.0,
        "filter_decompose": 16.0, "filter_recompose": 16.0,
        "filter_phi_analysis": 8.0 + 8.0 * K / n_ph,
        "filter_theta": 16.0 * K / n_ph,
        "filter_phi_synthesis": 8.0 + 8.0 * K / n_ph,
    }[cls]
    extra = 16 * 8 * npts if (cls == "rhs_stage" and n_v == 50) else 0
    return per_fp * fp + extra


def runs_of(shells):
    """(shell, count) of consecutive identical shells (one launch each)."""
    out = []
    for s in shells:
        if out and tuple(out[-1][0]) == tuple(s):
            out[-1][1] += 1
        else:
            out.append([tuple(s), 1])
    return out


LAUNCHES_PER_STEP = {"d_r": 4, "d_theta": 4, "d_phi": 4, "derivs_fused": 4, "rhs_stage": 4, "filter_decompose": 1,
                     "filter_phi_analysis": 1, "filter_theta": 1, "filter_phi_synthesis": 1, "filter_recompose": 1}


def step_bytes(shells, n_v, classes):
    return sum(LAUNCHES_PER_STEP[c] * bytes_per_launch(c, s, n_v, cnt) for c in classes for (s, cnt) in runs_of(shells))


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


def initial_state(g, shells, n_v, seed0, one_seed=False):
    """Seeded perturbed Kerr-Schild data on every shell (seed0 + shell index,
    or seed0 for all with one_seed: one smooth field across nested shells;
    gauge fields seed0 + 1000 + index), built by the library."""
    import numpy as np
    import torch
    from paper_1104_3408_amd import inputs
    g10, extra = [], []
    for k in range(len(shells)):
        r, th, ph = g.coords(k)
        g10.append(inputs.perturbed_kerr_schild(seed0 + (0 if one_seed else k), r, th, ph).ravel())
        if n_v == 58:
            dH, Q = inputs.gauge_perturbation(seed0 + 1000 + k, r, th, ph)
            extra.append(np.concatenate([dH, Q]).ravel())
    u = torch.zeros(g.state_size, dtype=torch.float64, device="cuda")
    ex = torch.from_numpy(np.concatenate(extra)).cuda() if extra else None
    g.kerr_schild_data(torch.from_numpy(np.concatenate(g10)).cuda(), u, extra8=ex)
    return u, g10


def class_representatives(shells):
    """Index of the first shell of every distinct shell size."""
    seen, out = set(), []
    for k, s in enumerate(shells):
        if tuple(s[:3]) not in seen:
            seen.add(tuple(s[:3]))
            out.append(k)
    return out


def run_form(shells, n_v, precision, steps, warmup, seed0, keep=(), filter="Yn", flags=0, one_seed=False):
    """One precision form of a workload: initial data, one step from it (the
    states of the shells in `keep` are returned on the host, for the error
    against the oracle), then warmup and `steps` timed steps (graph replay)."""
    import torch
    from paper_1104_3408_amd import shellspec as ss
    g = ss.ShellGrid(shells, n_fields=n_v, filter=filter, n_f=4, courant=4.0, precision=precision, flags=flags)
    u, g10 = initial_state(g, shells, n_v, seed0, one_seed)
    one = {}
    if keep:
        u1 = u.clone()
        g.rk_step(u1, 1)
        torch.cuda.synchronize()
        for k in keep:
            off, cnt, _ = g.info(k)
            one[k] = u1[off:off + cnt].cpu().numpy()
        del u1
    g.rk_step(u, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.rk_step(u, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fp = sum(n_v * a * b * c for (a, b, c, _, _) in shells)
    res = {"ms_per_step": 1e3 * (t1 - t0) / steps, "value": fp * steps / (t1 - t0), "steps": steps,
           "warmup": warmup, "state_finite": bool(torch.isfinite(u).all().item())}
    log("%s %s: %.3f ms/step" % (len(shells), PREC_NAMES[precision], res["ms_per_step"]))
    return res, g, u, g10, one


def err_stats(got, ref, u0):
    """max and RMS of got - ref relative to max|ref| and RMS ref, and the
    max relative to the change of the state max|ref - u0|."""
    import numpy as np
    d = got - ref
    return {"max_rel": float(np.abs(d).max() / np.abs(ref).max()),
            "rms_rel": float(np.sqrt(np.mean(d ** 2)) / np.sqrt(np.mean(ref ** 2))),
            "max_rel_to_change": float(np.abs(d).max() / max(np.abs(ref - u0).max(), 1e-300))}


def stored_oracle(case):
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "oracle_%s.npz" % case)
    return dict(np.load(path)) if os.path.exists(path) else None


def against_stored(case, precisions, steps_wanted=None):
    """Single-shell configuration run from the stored oracle evolution's seed
    and grid in each precision; error after each stored step count, on the
    stored sample, scaled by the oracle's full-state norms."""
    import numpy as np
    import torch
    from paper_1104_3408_amd import shellspec as ss
    ref = stored_oracle(case)
    if ref is None:
        return {"skipped": "no stored oracle evolution %s" % case}
    n_v, n_ph, n_th, n_r = [int(x) for x in ref["shape"]]
    r0, r1 = [float(x) for x in ref["radii"]]
    shells = [(n_r, n_th, n_ph, r0, r1)]
    idx = ref["idx"]
    saves = [int(n) for n in ref["steps"] if steps_wanted is None or n in steps_wanted]
    out = {"grid": "%dx%dx%d r[%g,%g], %d fields, seed %d" % (n_r, n_th, n_ph, r0, r1, n_v, int(ref["seed"]))}
    for prec in precisions:
        g = ss.ShellGrid(shells, n_fields=n_v, filter="Yn", n_f=4, courant=4.0, precision=prec)
        u, _ = initial_state(g, shells, n_v, int(ref["seed"]))
        u0 = u.cpu().numpy()[idx]
        assert abs(g.info(0)[2] - float(ref["dt"])) < 1e-15 * float(ref["dt"])
        e, done = {}, 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for n in saves:
            g.rk_step(u, n - done)
            done = n
            got = u.cpu().numpy()[idx]
            d = got - ref["vals_%d" % n]
            e["after_%d" % n] = {"max_rel": float(np.abs(d).max() / ref["max_u_%d" % n]),
                                 "rms_rel": float(np.sqrt(np.mean(d ** 2)) / ref["rms_u_%d" % n]),
                                 "max_rel_to_change": float(np.abs(d).max() / ref["max_du_%d" % n]),
                                 "rms_rel_to_change": float(np.sqrt(np.mean(d ** 2)) / ref["rms_du_%d" % n])}
        out[PREC_NAMES[prec]] = e
        g.close()
        del u
        log("%s %s against the stored oracle: %s" % (case, PREC_NAMES[prec], e))
    return out


def copy_bandwidth(mib=2048, reps=10):
    """Attainable HBM bandwidth on this machine: a device-to-device copy of `mib`
    MiB (as many bytes read as written), timed with HIP events; reads plus
    writes per second."""
    import torch
    src = torch.ones(mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        dst.copy_(src)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    out = {"GBps": 2 * src.numel() * 8 / ms / 1e6, "bytes_each_way": src.numel() * 8, "ms": ms,
           "frac_of_spec": 2 * src.numel() * 8 / ms / 1e6 / HBM_PEAK_GBS}
    del src, dst
    torch.cuda.empty_cache()
    return out


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


def oracle_steps(shells, keep, g10_all, dts, n_v=50):
    """The CPU oracle's filtered RK4 step (numpy FP64) of the shells in keep,
    from the same seeded metric the GPU started from.  Returns the states
    and the wall time of the steps alone."""
    import numpy as np
    from oracle.grid import Shell
    from oracle import initial_data as oid
    from oracle.evolve import Evolution
    states, secs, fp = {}, 0.0, 0
    for k in keep:
        n_r, n_th, n_ph, a, b = shells[k]
        sh = Shell(n_r, n_th, n_ph, a, b)
        u0 = oid.first_order_data(g10_all[k].reshape((10,) + sh.shape), sh)
        H, dH = oid.static_gauge(u0, sh)
        ev = Evolution(sh, n_v, H, dH, "Yn", 4)
        t0 = time.perf_counter()
        ref = ev.rk4_step(u0, dts[k])
        secs += time.perf_counter() - t0
        fp += n_v * sh.npts
        states[k] = (u0, ref)
    return states, secs, fp


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        return 1


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="batch64", choices=sorted(DESCRIPTIONS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true", help="skip the per-kernel HIP events")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the mixed-precision forms and the other configurations")
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
    seed0 = inputs.WORKLOAD_SEED[args.workload]
    reps = class_representatives(shells) if n_v == 50 else []
    log("workload %s: %d shells" % (args.workload, len(shells)))

    # headline: FP64, timed region = K filtered steps, one captured graph replayed
    res, g, u, g10, one64 = run_form(shells, n_v, ss.SG_PREC_FP64, args.steps, args.warmup, seed0, keep=reps)
    fp = sum(n_v * a * b * c for (a, b, c, _, _) in shells)
    dts = [g.info(k)[2] for k in range(len(shells))]
    graph_bytes = step_bytes(shells, n_v, ["derivs_fused", "rhs_stage", "filter_decompose", "filter_phi_analysis",
                                          "filter_theta", "filter_phi_synthesis", "filter_recompose"])
    out = {"metric": "field-points/s per filtered RK4 step", "value": res["value"], "unit": "field-points/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic", "config": {"workload": DESCRIPTIONS[args.workload], "name": args.workload,
                                          "shells": [list(s) for s in runs_of(shells)], "n_fields": n_v,
                                          "filter": "Yn", "n_f": 4, "courant": 4.0, "field_points": fp,
                                          "state_finite": res["state_finite"]},
           "step_roofline": {"bytes_per_step": graph_bytes, "achieved_GBps": graph_bytes / res["ms_per_step"] / 1e6,
                             "frac": graph_bytes / res["ms_per_step"] / 1e6 / HBM_PEAK_GBS,
                             "model": "algorithmic FP64 bytes of one step: derivatives 32 B per stage (u read "
                                      "once, three derivatives written, whether the graph runs them as one "
                                      "launch or three), rhs stage 56 B (+128 B per point of gauge), "
                                      "filter 16+16 B + spectral"}}
    if not args.no_timing:
        # second pass of K steps with HIP events around every launch on the
        # stream it runs on (eager launches; the three derivative contractions
        # of a stage then run as three separate launches, one class each)
        g.enable_timing(True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        g.rk_step(u, args.steps)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        ms, cnt = g.kernel_times()
        g.enable_timing(False)
        kern = {}
        for i, c in enumerate(ss.KERNEL_CLASSES):
            if not cnt[i]:
                continue
            byts = args.steps * step_bytes(shells, n_v, [c])
            kern[c] = {"total_ms": ms[i], "launches": cnt[i], "avg_us": 1e3 * ms[i] / cnt[i],
                       "bytes_per_launch": byts / cnt[i], "GBps": byts / ms[i] / 1e6,
                       "frac_hbm": byts / ms[i] / 1e6 / HBM_PEAK_GBS}
        dom = max(kern, key=lambda c: kern[c]["total_ms"])
        k = kern[dom]
        out["roofline"] = {"kernel": dom, "bound": "hbm", "achieved": k["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": k["frac_hbm"], "traffic": profiled_traffic(args.workload, dom),
                           "bytes_per_launch": k["bytes_per_launch"], "avg_launch_us": k["avg_us"]}
        out["kernels"] = kern
        out["timing_pass_ms_per_step"] = 1e3 * (t3 - t2) / args.steps
        log("timing pass done, dominant kernel %s %.2f us" % (dom, k["avg_us"]))
    if args.copy_probe_mb:
        src = torch.empty(args.copy_probe_mb * (1 << 20) // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes_each_way"] = src.numel() * 8
        del src, dst
    g.close()
    del u, g
    torch.cuda.empty_cache()

    ones = {"fp64": one64}
    if not args.no_variants:
        out["measured_copy_bandwidth"] = copy_bandwidth()
        log("copy bandwidth %.0f GB/s" % out["measured_copy_bandwidth"]["GBps"])
        var = {}
        for prec in (ss.SG_PREC_FP32, ss.SG_PREC_BF16X3):
            r, gm, um, _, onem = run_form(shells, n_v, prec, args.steps, args.warmup, seed0, keep=reps)
            r["speedup_vs_fp64"] = r["value"] / res["value"]
            var[PREC_NAMES[prec]] = r
            ones[PREC_NAMES[prec]] = onem
            gm.close()
            del um, gm
            torch.cuda.empty_cache()
        out["mixed_forms"] = var
        best = max(var, key=lambda p: var[p]["value"])
        out["best_mixed"] = {"form": best, "value": var[best]["value"], "ms_per_step": var[best]["ms_per_step"],
                             "speedup_vs_fp64": var[best]["speedup_vs_fp64"]}
        other = {}
        if args.workload != "ks49":
            s49 = inputs.workload_shells("ks49")[0]
            other["ks49"] = {"description": DESCRIPTIONS["ks49"]}
            for prec in (ss.SG_PREC_FP64, ss.SG_PREC_FP32, ss.SG_PREC_BF16X3):
                r, gm, um, _, _ = run_form(s49, 50, prec, args.steps, args.warmup, inputs.WORKLOAD_SEED["ks49"])
                other["ks49"][PREC_NAMES[prec]] = r
                gm.close()
                del um, gm
            other["ks49"]["error_vs_stored_oracle"] = against_stored(
                "shell49_100", (ss.SG_PREC_FP64, ss.SG_PREC_FP32, ss.SG_PREC_BF16X3))
        if args.workload != "ks33":
            s33 = inputs.workload_shells("ks33")[0]
            r, gm, um, _, _ = run_form(s33, 50, ss.SG_PREC_FP64, args.steps, args.warmup, inputs.WORKLOAD_SEED["ks33"])
            other["ks33"] = {"description": DESCRIPTIONS["ks33"], "fp64": r,
                             "error_vs_stored_oracle": against_stored("shell33_100", (ss.SG_PREC_FP64,))}
            gm.close()
            del um, gm
        if args.workload != "large8":
            s8, nv8 = inputs.workload_shells("large8")
            other["large8"] = {"description": DESCRIPTIONS["large8"]}
            for prec in (ss.SG_PREC_FP64, ss.SG_PREC_FP32, ss.SG_PREC_BF16X3):
                r, gm, um, _, _ = run_form(s8, nv8, prec, 10, 2, inputs.WORKLOAD_SEED["large8"])
                other["large8"][PREC_NAMES[prec]] = r
                gm.close()
                del um, gm
                torch.cuda.empty_cache()
        # beside the hot path, measured: nested shells (four 33x32x64 shells
        # on [1.8, 17.8] coupled at their shared spheres against the same four
        # shells uncoupled) and the scalar Y and graded Yg filters on the
        # 33x32x64 shell against Yn
        nest = [(33, 32, 64, 1.8 + 4.0 * k, 5.8 + 4.0 * k) for k in range(4)]
        other["nested4"] = {"description": "4 perturbed Kerr-Schild shells 33x32x64 on [1.8, 5.8, 9.8, 13.8, 17.8], "
                                           "50 fields, Yn n_f=4, FP64, one time step for the chain"}
        for name, flags in (("coupled", ss.SG_NESTED), ("independent", 0)):
            r, gm, um, _, _ = run_form(nest, 50, ss.SG_PREC_FP64, args.steps, args.warmup, 7000, flags=flags,
                                       one_seed=True)
            other["nested4"][name] = r
            gm.close()
            del um, gm
        s33 = inputs.workload_shells("ks33")[0]
        other["filters_33"] = {"description": DESCRIPTIONS["ks33"] + ", filter kind varied"}
        for kind in ("Y", "Yg"):
            r, gm, um, _, _ = run_form(s33, 50, ss.SG_PREC_FP64, args.steps, args.warmup,
                                       inputs.WORKLOAD_SEED["ks33"], filter=kind)
            other["filters_33"][kind] = r
            gm.close()
            del um, gm
        torch.cuda.empty_cache()
        out["other_configs"] = other
        out["fft_vs_matmul_dphi"] = fft_vs_matmul()
        log("FFT comparison done")

    if not args.no_cpu_baseline and reps:
        log("oracle steps on the host, all cores (%d threads)" % blas_threads())
        states, secs, fp_s = oracle_steps(shells, reps, g10, dts)
        desc = ", ".join("%dx%dx%d" % tuple(shells[k][:3]) for k in reps)
        out["cpu_baseline"] = {"value": fp_s / secs, "unit": "field-points/s", "cores": int(blas_threads()),
                               "kind": "oracle", "cpu": cpu_model(),
                               "sample": "1 filtered RK4 step of one shell per size class (%s; %d field-points), "
                                         "%.1f s" % (desc, fp_s, secs)}
        errs = {}
        for form, st in ones.items():
            errs[form] = {"%dx%dx%d" % tuple(shells[k][:3]): err_stats(st[k].reshape(states[k][1].shape),
                                                                       states[k][1], states[k][0]) for k in reps}
        out["error_vs_oracle_after_1_step"] = errs
        try:
            from threadpoolctl import threadpool_limits
            small = reps[:2]
            with threadpool_limits(limits=1):
                _, s1, f1 = oracle_steps(shells, small, g10, dts)
            out["cpu_baseline_1core"] = {
                "value": f1 / s1, "unit": "field-points/s", "cores": 1, "kind": "oracle", "cpu": cpu_model(),
                "sample": "1 filtered RK4 step of the %s shells, BLAS limited to one thread, %.1f s"
                          % (", ".join("%dx%dx%d" % tuple(shells[k][:3]) for k in small), s1)}
        except ImportError:
            pass
        log("oracle done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
