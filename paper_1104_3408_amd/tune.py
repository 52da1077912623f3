"""Autotuner of the library's tile shapes (runs on the GPU).

For every shell size of the benchmark workloads and every precision mode it
times the candidate tile shapes of each contraction kernel class with HIP
events (the library's timing mode: eager launches, one kernel class each) on
a batch of identical shells as the workloads run them and keeps the fastest
per class.  Whole captured steps then decide what per-class timings cannot
see: the three derivative contractions of a stage as one launch (which needs
their workgroups to agree) or as three launches on forked streams, the d_theta
tile inside them, and the tuned shapes against the defaults (--forms-only
makes only this choice, on the shapes of an existing table).  The result is a
text table, one line per (N_r, N_theta, n_fields, precision), read by
shell_grid_create (see csrc/tuning.cpp):

  python -m paper_1104_3408_amd.tune [--out paper_1104_3408_amd/tuning.txt] [--classes 17,25,33,49,65]
                                     [--precisions 0,1,2] [--merge] [--forms-only]

Candidate values are target rows per wave (blocked_shape turns a target into
rows per wave and 8, 12 or 16 waves per workgroup; targets giving the same
shape are timed once), 4, 8 or 16 waves per workgroup for the theta filter,
the d_phi form (circulant window or parity) and, in FP64, the d_theta tile
(64 columns or a meridian plane pair) and the circulant d_phi on the matrix
cores or the vector units.
"""
import argparse
import os
import sys
import tempfile
import time

HERE = os.path.dirname(os.path.abspath(__file__))
FIELDS = ["dr_rows", "th_rows", "dph_rows", "ana_rows", "syn_rows", "filt_waves", "dph_par", "th_plane", "fuse",
          "dph_mfma"]
DEFAULT = {"dr_rows": 9, "th_rows": 4, "dph_rows": 8, "ana_rows": 8, "syn_rows": 8, "filt_waves": 8, "dph_par": -1,
           "th_plane": 0, "fuse": 1, "dph_mfma": 0}
# kernel class (KERNEL_CLASSES order of the binding) timed for each field
FIELD_CLASS = {"dr_rows": "d_r", "th_rows": "d_theta", "dph_rows": "d_phi", "ana_rows": "filter_phi_analysis",
               "syn_rows": "filter_phi_synthesis", "filt_waves": "filter_theta", "dph_par": "d_phi",
               "th_plane": "d_theta", "dph_mfma": "d_phi"}
ROW_TARGETS = (3, 4, 5, 6, 8, 9, 11, 13, 16)
# shell sizes of the workloads: (N_r, N_theta, n_fields, shells per batch, r_max)
CLASSES = {17: (17, 16, 50, 16, 11.8), 25: (25, 24, 50, 16, 11.8), 33: (33, 32, 50, 16, 11.8),
           49: (49, 48, 50, 16, 11.8), 65: (65, 64, 58, 8, 21.8)}


def blocked_shape(n_out, target, k_min=8, k_max=16, max_rows=20):
    """Rows per wave and waves per workgroup the library derives from a
    target (the host rule of csrc/derivs.hip blocked_shape)."""
    nw = -(-n_out // target)
    nw = -(-nw // 4) * 4
    nw = min(max(nw, k_min), k_max)
    R = -(-n_out // nw)
    return (R, nw) if R <= max_rows else None


def dph_parity(tune, prec):
    """Whether the library builds d_phi in the parity form (tuning value -1:
    parity in the FP32 mode only)."""
    return tune["dph_par"] == 1 if tune["dph_par"] >= 0 else prec == 1


def write_table(path, entries):
    with open(path, "w") as f:
        f.write("# n_r n_theta n_fields precision " + " ".join(FIELDS) + "\n")
        for (n_r, n_th, n_v, prec), t in sorted(entries.items()):
            f.write("%d %d %d %d %s\n" % (n_r, n_th, n_v, prec, " ".join(str(t[k]) for k in FIELDS)))


def read_table(path):
    """Entries of an existing table (missing file: none)."""
    out = {}
    if not os.path.exists(path):
        return out
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x) for x in line.split()]
        t = dict(DEFAULT)
        t.update(zip(FIELDS, v[4:]))
        out[tuple(v[:4])] = t
    return out


def log(msg):
    print("[tune %7.1fs] %s" % (time.perf_counter() - T0, msg), file=sys.stderr, flush=True)


T0 = time.perf_counter()


def measure(key, tune, table_path, steps=4, graph=False):
    """Per-class eager kernel times (ms per step) or the captured step time
    of a batch of identical shells with the given tile shapes."""
    import numpy as np
    import torch
    from . import shellspec as ss
    from . import inputs
    n_r, n_th, n_v, prec = key
    _, _, _, count, r1 = CLASSES[n_r]
    write_table(table_path, {key: tune})
    shells = [(n_r, n_th, 2 * n_th, 1.8, r1)] * count
    g = ss.ShellGrid(shells, n_fields=n_v, precision=prec)
    r, th, ph = g.coords(0)
    g10 = np.tile(inputs.perturbed_kerr_schild(7, r, th, ph).ravel(), count)
    u = torch.zeros(g.state_size, dtype=torch.float64, device="cuda")
    extra = torch.zeros(8 * g.n_points, dtype=torch.float64, device="cuda") if n_v == 58 else None
    g.kerr_schild_data(torch.from_numpy(g10).cuda(), u, extra8=extra)
    g.rk_step(u, 1)
    torch.cuda.synchronize()
    if graph:
        g.rk_step(u, 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.rk_step(u, steps)
        torch.cuda.synchronize()
        out = 1e3 * (time.perf_counter() - t0) / steps
    else:
        g.enable_timing(True)
        g.rk_step(u, steps)
        ms, _ = g.kernel_times()
        g.enable_timing(False)
        out = {c: ms[i] / steps for i, c in enumerate(ss.KERNEL_CLASSES)}
    g.close()
    del u
    torch.cuda.empty_cache()
    return out


def tune_class(key, table_path):
    n_r, n_th, n_v, prec = key
    # rows each field's target applies to: radial points, theta rows of the
    # equator-parity form, phi rows (circulant d_phi) or row pairs (parity
    # forms: m <= m_keep for the analysis, j <= N_phi / 2 otherwise)
    m_keep = n_th - 1 - 4

    def n_out(field, tune):
        return {"dr_rows": n_r, "th_rows": (n_th + 1) // 2,
                "dph_rows": n_th + 1 if dph_parity(tune, prec) else 2 * n_th,
                "ana_rows": m_keep + 1, "syn_rows": n_th + 1}[field]
    best = dict(DEFAULT)
    memo = {}

    def timed(trial):
        k = tuple(trial[f] for f in FIELDS)
        if k not in memo:
            memo[k] = measure(key, trial, table_path)
        return memo[k]
    report = {}
    # the d_phi form first: it decides what dph_rows counts
    for field in ["dph_par"] + [f for f in FIELDS if f not in ("dph_par", "fuse")]:
        cls = FIELD_CLASS[field]
        if field == "filt_waves":
            cands = [4, 8, 16]
        elif field == "dph_par":
            cands = [0, 1]
        elif field == "th_plane":
            cands = [0, 1] if prec == 0 else [0]     # the plane tile is the FP64 form
        elif field == "dph_mfma":                    # FP64 circulant d_phi on the matrix cores
            cands = [0, 1] if prec == 0 and (2 * n_th) % 16 == 0 and not dph_parity(best, prec) else [0]
        else:
            shapes = {}
            for t in ROW_TARGETS:
                sh = blocked_shape(n_out(field, best), t)
                if sh is not None and sh not in shapes:
                    shapes[sh] = t
            cands = sorted(shapes.values())
        times = {}
        for v in cands:
            trial = dict(best)
            trial[field] = v
            times[v] = timed(trial)[cls]
        v_best = min(times, key=times.get)
        best[field] = v_best
        report[field] = {str(v): round(t, 4) for v, t in times.items()}
        log("%s %s: %s -> %s" % (key, field, report[field], v_best))
    graph = choose_forms(key, best, table_path)
    return graph["best"], {"per_class_ms": report, "graph_ms": graph["graph_ms"]}


def choose_forms(key, tuned, table_path):
    """Whole captured steps decide what the per-class timings cannot see:
    the one-launch form of the three derivative contractions against three
    launches on forked streams (fuse), the d_theta tile inside each, and the
    tuned shapes against the defaults."""
    prec = key[3]
    cands = {"tuned": dict(tuned, fuse=1), "tuned, three launches": dict(tuned, fuse=0),
             "defaults": dict(DEFAULT)}
    if prec == 0:
        flip = 1 - tuned["th_plane"]
        cands["tuned, other theta tile"] = dict(tuned, fuse=1, th_plane=flip)
        cands["tuned, three launches, other theta tile"] = dict(tuned, fuse=0, th_plane=flip)
    graph_ms, seen = {}, {}
    for name, t in cands.items():
        k = tuple(t[f] for f in FIELDS)
        if k not in seen:
            seen[k] = measure(key, t, table_path, steps=6, graph=True)
        graph_ms[name] = round(seen[k], 4)
    name = min(graph_ms, key=graph_ms.get)
    log("%s graph step ms: %s -> %s" % (key, graph_ms, name))
    return {"best": cands[name], "graph_ms": graph_ms}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "tuning.txt"))
    ap.add_argument("--classes", default="17,25,33,49,65")
    ap.add_argument("--precisions", default="0,1,2")
    ap.add_argument("--merge", action="store_true", help="keep the other entries of an existing table")
    ap.add_argument("--forms-only", action="store_true",
                    help="keep the tile shapes of the existing table and only choose the forms by step time")
    args = ap.parse_args()
    import json
    entries, details = {}, {}
    old = read_table(args.out) if args.merge else {}
    fd, tmp = tempfile.mkstemp(suffix=".txt", prefix="sg_tune_")
    os.close(fd)
    os.environ["SG_TUNING_FILE"] = tmp
    try:
        for prec in [int(p) for p in args.precisions.split(",")]:
            for c in [int(x) for x in args.classes.split(",")]:
                n_r, n_th, n_v, _, _ = CLASSES[c]
                key = (n_r, n_th, n_v, prec)
                if args.forms_only:
                    r = choose_forms(key, read_table(args.out).get(key, dict(DEFAULT)), tmp)
                    entries[key], details[str(key)] = r["best"], {"graph_ms": r["graph_ms"]}
                else:
                    entries[key], details[str(key)] = tune_class(key, tmp)
                write_table(args.out, {**old, **entries})     # progress survives an interrupted run
    finally:
        os.unlink(tmp)
        del os.environ["SG_TUNING_FILE"]
    write_table(args.out, {**old, **entries})
    print(json.dumps(details))


if __name__ == "__main__":
    main()
