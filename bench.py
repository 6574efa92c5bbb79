"""Benchmark: alpha complex of a 3,000,000-atom synthetic capsid shell on one MI355X.

One step = one full alpha-complex build through the C ABI from device-resident
inputs (quantise, grid binning, candidate edges / triangles / tetrahedra,
pruning, Size propagation, sorted output on the device). Prints one JSON line.

The same line carries two secondary workloads (skip them with --no-extras):
  "batch": 512 molecules of 500-50,000 atoms in one batched call (cell sides
           from the autotuner), against 512 sequential single-molecule calls;
  "union_measure": 64 jittered frames of the 100k-atom molecule, union volume
           and area forward + backward, per frame and as one batch.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-extras]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X FP64 vector

KERNEL_OF_STAGE = {
    "neighbours_count": "k_neighbours<0, 16, true>",
    "neighbours_fill": "k_nbr_compact<16>",
    "triangles_count": "k_triangles<0, true>",
    "triangles_fill": "k_tri_compact",
    "triangles_ac2_tetrahedra": "k_tet_candidates<0, true>",
    "tetrahedra_fill": "k_tet_compact",
    "tetrahedra_ac2": "k_tet_ac2",
    "triangles_final": "k_tri_final",
    "edges_final": "k_edge_final",
    "vertices_final": "k_vert_final",
}
KERNEL_SOURCES = ["paper_1908_05944_amd/csrc/kernels.hpp", "paper_1908_05944_amd/csrc/predicates.hpp",
                  "paper_1908_05944_amd/csrc/common.hpp", "paper_1908_05944_amd/csrc/radix.hpp",
                  "paper_1908_05944_amd/csrc/measure.hpp", "paper_1908_05944_amd/csrc/sweep.hpp",
                  "paper_1908_05944_amd/csrc/partition.hpp", "paper_1908_05944_amd/csrc/emit.hpp",
                  "paper_1908_05944_amd/csrc/alphacx.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_3Mshell.json")
VALU_FILE = os.path.join(ROOT, "profiles", "valu_3Mshell.json")
# vector lane-operations per second at the issue limit: 256 CUs x 4 SIMDs x
# 16 lanes x 2.4 GHz (a float64 FMA issues at this rate: 78.6 TFLOP/s)
VALU_ISSUE_PEAK_T = 256 * 4 * 16 * 2.4e9 / 1e12


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _profile_record(path):
    """A committed rocprofv3 counter summary (JSON), or None if it is missing
    or was taken on other kernel sources."""
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    return rec if rec.get("source_sha") == kernel_source_hash() else None


def measured_traffic(stage):
    """HBM bytes per launch of the stage's kernel (FETCH_SIZE + WRITE_SIZE,
    calibrated), or None."""
    rec = _profile_record(TRAFFIC_FILE)
    k = None if rec is None else rec.get("kernels", {}).get(KERNEL_OF_STAGE.get(stage, stage))
    return None if k is None else k.get("traffic_bytes")


def measured_traffic_total():
    """HBM bytes of one whole build (every kernel's per-launch traffic times its
    launches per build), or None."""
    rec = _profile_record(TRAFFIC_FILE)
    if rec is None or "builds" not in rec:
        return None
    return sum(k["traffic_bytes"] * k["launches"] for k in rec["kernels"].values()) / rec["builds"]


def measured_valu_lane_ops(stage):
    """Vector lane-operations per launch of the stage's kernel (VALU wave
    instructions x 64, from the committed SQ counters), or None."""
    rec = _profile_record(VALU_FILE)
    k = None if rec is None else rec.get("kernels", {}).get(KERNEL_OF_STAGE.get(stage, stage))
    return None if k is None else k.get("valu_lane_ops_per_launch")


def neighbour_pairs_tested(X, W, aq, cell_mA):
    """P_e: ball pairs the neighbour pass tests, replicating its grid on the
    host (cell side, growth rule and reach as the build takes them; every ball
    of each scanned cell row whose slab lies within 2 s_g of the ball)."""
    import numpy as np
    X = X.astype(np.int64)
    n = len(X)
    sg2 = max(int(W.max()) + aq, 0)
    sgc = math.isqrt(sg2)
    sgc += sgc * sgc < sg2
    lo = X.min(0)
    ext = X.max(0) - lo + 1
    side = cell_mA if cell_mA > 0 else max(sgc, 1)
    nc = lambda sd: int(np.prod((ext + sd - 1) // sd))
    while nc(side) > max(8 * n, 1 << 22):
        side = side + side // 4 + 1
    nx, ny, nz = [int(v) for v in (ext + side - 1) // side]
    reach = (2 * sgc + side - 1) // side
    c = (X - lo) // side
    cid = (c[:, 2] * ny + c[:, 1]) * nx + c[:, 0]
    cs = np.concatenate([[0], np.cumsum(np.bincount(cid, minlength=nx * ny * nz))])
    lim, reach1 = 4 * sg2, 2 * sgc
    x0 = np.maximum(c[:, 0] - reach, 0)
    x1 = np.minimum(c[:, 0] + reach, nx - 1)
    total = 0
    for dz in range(-reach, reach + 1):
        z = c[:, 2] + dz
        zlo = lo[2] + z * side
        dzm = np.where(X[:, 2] < zlo, zlo - X[:, 2], np.where(X[:, 2] > zlo + side - 1, X[:, 2] - zlo - side + 1, 0))
        okz = (z >= 0) & (z < nz) & (dzm <= reach1) & (lim - dzm * dzm >= 0)
        for dy in range(-reach, reach + 1):
            y = c[:, 1] + dy
            ylo = lo[1] + y * side
            dym = np.where(X[:, 1] < ylo, ylo - X[:, 1], np.where(X[:, 1] > ylo + side - 1, X[:, 1] - ylo - side + 1, 0))
            ok = okz & (y >= 0) & (y < ny) & (dym <= reach1) & (lim - dzm * dzm - dym * dym >= 0)
            rb = (np.clip(z, 0, nz - 1) * ny + np.clip(y, 0, ny - 1)) * nx
            total += int(np.sum(np.where(ok, cs[rb + x1 + 1] - cs[rb + x0], 0)))
    return total, nx * ny * nz


def algorithmic_work(n, C, E, F, Q, K, Nn, Pe):
    """Algorithmic HBM bytes and float64 operations of one build and of its
    single-kernel stages, from measured counts (balls n, grid cells C,
    candidate edges E, triangles F and tetrahedra Q, output counts K[d],
    neighbour entries Nn, pairs tested Pe). Bytes: inputs read once, every
    candidate list written once and read once, the output written once; the
    int32 quantised balls (16 B), sorted balls and order (36 B), cell table
    (8 B per cell), candidates 8 / 12 / 16 B, output rows 4 (d + 1) + 8 B.
    Operations: 12 per pair tested, 40 per triple and 80 per quadruple (the
    examined triples and quadruples are at least the candidates, which are
    counted here), plus per candidate its ortho-centre setup (30 / 60 / 120)
    and 12 per neighbour of its AC2 scan (nbr = Nn / n neighbours on average)."""
    nbr = Nn / n
    out = sum(K[d] * (4 * (d + 1) + 8) for d in range(4))
    B = 16 * n + 36 * n + 8 * C + 2 * (8 * E + 12 * F + 16 * Q) + out
    FL = 12 * Pe + 40 * F + 80 * Q + E * (30 + 12 * nbr) + F * (60 + 12 * nbr) + Q * (120 + 12 * nbr)
    stage_bytes = {
        "neighbours_count": 16 * n + 8 * C + 8 * E,
        "neighbours_fill": 2 * 8 * E,
        "triangles_count": 16 * n + 8 * E + 12 * F,
        "triangles_fill": 2 * 12 * F,
        "triangles_ac2_tetrahedra": 16 * n + 12 * F + 16 * Q,
        "tetrahedra_fill": 2 * 16 * Q,
        "tetrahedra_ac2": 16 * n + 16 * Q + 24 * K[3],
        "triangles_final": 12 * F + 20 * K[2],
        "edges_final": 8 * E + 16 * K[1],
        "vertices_final": 16 * n + 12 * K[0],
    }
    stage_flops = {
        "neighbours_count": 12 * Pe + 12 * Nn,
        "triangles_count": 40 * F + E * (30 + 12 * nbr),
        "triangles_ac2_tetrahedra": 80 * Q + F * (60 + 12 * nbr),
        "tetrahedra_ac2": Q * (120 + 12 * nbr),
    }
    return B, FL, stage_bytes, stage_flops


def host_cpu():
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count()
    return {"nproc": os.cpu_count(), "available_to_process": avail, "cpu_model": model}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _timed(torch, fn, reps):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def bench_partition(acx, torch, log, xyz, rad, opts, host_xyz, host_rad, reps=3):
    """Partitioned builds of the 3M-atom shell (slabs along x with a halo):
    device-resident (inputs and results on the device) against the single
    device build, and streamed from host memory (one slab on the device at a
    time, results back on the host) against the single host-array build."""
    out, out_host = {}, {}
    for parts in (4, 16):
        acx.ac_alpha_complex_partitioned(xyz, rad, 0.0, parts, options=opts).close()
        t = _timed(torch, lambda: acx.ac_alpha_complex_partitioned(xyz, rad, 0.0, parts, options=opts).close(), reps)
        out[str(parts)] = t * 1e3
        t = _timed(torch, lambda: acx.ac_alpha_complex_partitioned_host(host_xyz, host_rad, 0.0, parts,
                                                                        options=opts).close(), 1)
        out_host[str(parts)] = t * 1e3
    log("[bench] partitioned: " + ", ".join(f"{p} slabs {v:.2f} ms" for p, v in out.items())
        + "; from host memory: " + ", ".join(f"{p} slabs {v:.1f} ms" for p, v in out_host.items()))
    return {"metric": "partitioned build ms", "unit": "ms per build", "higher_is_better": False, "ms_by_slabs": out,
            "host_streamed_ms_by_slabs": out_host,
            "config": {"workload": "3M-atom shell, alpha = 0, slabs of equal width along x; host-streamed: host "
                                   "arrays in and out, one slab on the device at a time"}}


def bench_cell_order(acx, torch, log, xyz, rad, opts, reps=5):
    """The 3M-atom build with grid cells numbered along a Morton curve against
    row-major numbering (same cell side): whole-build time and the per-stage
    device times, which show where memory locality changes the cost."""
    out = {}
    for name, order in (("row_major", 0), ("morton", 1)):
        o = dict(opts, cell_order=order)
        acx.ac_alpha_complex_device(xyz, rad, 0.0, options=o).close()
        t = _timed(torch, lambda: acx.ac_alpha_complex_device(xyz, rad, 0.0, options=o).close(), reps)
        stages = {}
        for _ in range(3):
            c = acx.ac_alpha_complex_device(xyz, rad, 0.0, options=dict(o, profile=1))
            for k, v in c.stage_ms().items():
                stages[k] = stages.get(k, 0.0) + v / 3
            c.close()
        out[name] = {"ms_per_build": t * 1e3, "stage_ms": stages}
    log(f"[bench] cell order: row-major {out['row_major']['ms_per_build']:.3f} ms, "
        f"Morton {out['morton']['ms_per_build']:.3f} ms per build")
    return {"metric": "build ms by cell order", "unit": "ms per build", "higher_is_better": False, **out,
            "config": {"workload": "3M-atom shell, alpha = 0, same cell side, row-major vs Morton cell numbering"}}


def bench_sweep(acx, torch, log, xyz, rad, opts, reps=3):
    """Alpha sweep on the 3M-atom shell: the complexes at alpha = 0, 0.25, ...,
    2 A^2 from one ac_alpha_sweep_device call against one direct build per
    value (the results are identical; the tests check that)."""
    alphas = [0.25 * k for k in range(9)]

    def sweep():
        for c in acx.ac_alpha_sweep_device(xyz, rad, alphas, options=opts):
            c.close()

    def direct():
        for a in alphas:
            acx.ac_alpha_complex_device(xyz, rad, a, options=opts).close()

    sweep()
    t_sweep = _timed(torch, sweep, reps)
    t_direct = _timed(torch, direct, reps)
    cs = acx.ac_alpha_sweep_device(xyz, rad, [alphas[-1]], options=opts)
    top = cs[0].counts()
    cs[0].close()
    log(f"[bench] sweep: {len(alphas)} alpha values in {t_sweep * 1e3:.2f} ms as one sweep, "
        f"{t_direct * 1e3:.2f} ms as direct builds ({t_direct / t_sweep:.2f}x)")
    return {
        "metric": "alpha sweep ms",
        "value": t_sweep * 1e3,
        "unit": "ms for the whole sweep",
        "higher_is_better": False,
        "direct_builds_ms": t_direct * 1e3,
        "speedup_vs_direct": t_direct / t_sweep,
        "counts_at_alpha_max": top,
        "config": {"workload": "3M-atom shell, alpha = 0, 0.25, ..., 2 A^2 (9 values)", "alphas": alphas},
    }


# Table 2 of the paper splits a build into eight categories. The per-step
# arrangement of a profiled build (profile = stage count + 2) runs the AC2
# tests of candidate edges and triangles as kernels of their own, so they
# fall into the paper's pruning categories; vertices (not timed in the paper)
# are counted with the edges. "output" (sorting the result by input ids) has
# no category there.
TABLE2_CATEGORIES = {
    "grid": ["quantise", "binning"],
    "potential_edges": ["neighbours_count", "neighbours_scan", "neighbours_fill"],
    "potential_triangles": ["triangles_count", "triangles_scan", "triangles_fill"],
    "potential_tetrahedra": ["triangles_ac2_tetrahedra", "tetrahedra_scan", "tetrahedra_fill"],
    "ac2_tetrahedra": ["tetrahedra_ac2"],
    "ac2_triangles": ["triangles_ac2", "triangles_final"],
    "ac2_edges_vertices": ["edges_ac2", "edges_final", "vertices_final"],
    "output": ["emit"],
}


def bench_table2(acx, synth, torch, log, reps=5):
    """Per-stage split in the categories of the paper's Table 2 on synthetic
    molecules of the sizes of its PDB molecules (seeds 500 + k), alpha = 0, 1
    and 2 A^2. Stage times are HIP events of profiled builds in the per-step
    arrangement (median of `reps`); "memory" is the host-array call minus the
    device-array call (inputs up, every result array down)."""
    import numpy as np
    split = len(acx.stage_names()) + 2
    sizes = [260, 1505, 1509, 4384, 8142, 16068, 16647, 58674]
    rows = []
    for k, n in enumerate(sizes):
        m = synth.molecule(n, 500 + k)
        X = torch.from_numpy(m.xyz).cuda()
        R = torch.from_numpy(m.radii).cuda()
        for alpha in (0.0, 1.0, 2.0):
            acx.ac_alpha_complex_device(X, R, alpha).close()
            stages = []
            for _ in range(reps):
                c = acx.ac_alpha_complex_device(X, R, alpha, options={"profile": split})
                stages.append(c.stage_ms())
                counts = c.counts()
                c.close()
            t_dev = _timed(torch, lambda: acx.ac_alpha_complex_device(X, R, alpha).close(), reps)
            t_host = _timed(torch, lambda: acx.ac_alpha_complex(m.xyz, m.radii, alpha).close(), reps)
            # the same build recorded once and replayed as a HIP graph (no host
            # synchronisation inside; the result stays in the plan's buffers)
            try:
                plan = acx.Plan(X, R, np.array([0, n]), alpha)
            except acx.AlphaCxError:  # a stage needs the counted fill: no recorded build
                plan = None
            t_rec = None
            if plan is not None:
                plan.launch()
                plan.result().close()
                t_rec = _timed(torch, plan.launch, reps)
                plan.close()
            med = {key: float(np.median([max(st[key], 0.0) for st in stages])) for key in stages[0]}
            cat = {name: sum(med[x] for x in parts) for name, parts in TABLE2_CATEGORIES.items()}
            cat["memory"] = max(t_host - t_dev, 0.0) * 1e3
            rows.append({"atoms": n, "alpha": alpha, "simplices": sum(counts), "device_ms": t_dev * 1e3,
                         "recorded_replay_ms": None if t_rec is None else t_rec * 1e3,
                         "ms": {key: round(v, 4) for key, v in cat.items()}})
    est = ["potential_edges", "potential_triangles", "potential_tetrahedra"]
    pru = ["ac2_tetrahedra", "ac2_triangles", "ac2_edges_vertices"]  # Steps 2-5
    share = {}
    for name, parts in (("memory_grid", ["memory", "grid"]), ("estimation", est), ("pruning", pru),
                        ("ac2_tetrahedra", ["ac2_tetrahedra"]), ("output", ["output"])):
        share[name] = float(np.mean([sum(r["ms"][x] for x in parts) / sum(r["ms"].values()) for r in rows]))
    for r in rows:
        log(f"[bench] table2: {r['atoms']:6d} atoms alpha {r['alpha']:.1f}: {r['device_ms']:.3f} ms device "
            f"({r['recorded_replay_ms'] or float('nan'):.3f} ms as a graph replay), "
            + ", ".join(f"{key} {v:.3f}" for key, v in r["ms"].items()))
    log("[bench] table2 mean shares: " + ", ".join(f"{key} {v:.2f}" for key, v in share.items()))
    return {"rows": rows, "mean_share": share,
            "config": {"workload": "synthetic molecules of the paper's Table 1-2 sizes, alpha = 0, 1, 2 A^2",
                       "categories": TABLE2_CATEGORIES}}


def bench_batch(acx, synth, torch, log, reps=5):
    """512 molecules, sizes log-uniform in [500, 50000] atoms (seed 999), one
    batched call against 512 sequential single-molecule calls."""
    import numpy as np
    t0 = time.time()
    sizes = synth.batch_sizes()
    mols = [synth.molecule(int(k), 1000 + i) for i, k in enumerate(sizes)]
    xyz = np.concatenate([m.xyz for m in mols])
    rad = np.concatenate([m.radii for m in mols])
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    log(f"[bench] batch: {len(mols)} molecules, {len(rad)} atoms generated in {time.time() - t0:.1f} s")
    X = torch.from_numpy(xyz).cuda()
    R = torch.from_numpy(rad).cuda()
    t0 = time.perf_counter()
    cells, buckets = acx.ac_tune_cells(X, R, off, 0.0)
    tune_s = time.perf_counter() - t0
    per_bucket = {int(b): int(cells[np.nonzero(buckets == b)[0][0]]) for b in np.unique(buckets)}
    log(f"[bench] batch: tuner {tune_s:.2f} s, cell side (mA) per size bucket {per_bucket}")

    def batched(cell=None):
        acx.ac_alpha_complex_batch(X, R, off, 0.0, cell_mA=cell).close()

    def sequential():
        for m in range(len(mols)):
            a, b = int(off[m]), int(off[m + 1])
            acx.ac_alpha_complex_device(X[a:b], R[a:b], 0.0).close()

    batched(cells)
    sequential()
    t_tuned = _timed(torch, lambda: batched(cells), reps)
    t_default = _timed(torch, lambda: batched(None), reps)
    t_seq = _timed(torch, sequential, 1)
    c = acx.ac_alpha_complex_batch(X, R, off, 0.0, cell_mA=cells)
    counts = c.counts()
    c.close()
    # the same batch as a recorded build: one HIP graph replay per batch (no
    # host synchronisation inside), and replay + result (counts read back,
    # rows copied into a new result)
    t0 = time.perf_counter()
    plan = acx.Plan(X, R, off, 0.0, cell_mA=cells)
    plan_s = time.perf_counter() - t0
    plan.launch()
    plan.result().close()
    t_replay = _timed(torch, plan.launch, reps)

    def replay_result():
        plan.launch()
        plan.result().close()

    t_replay_res = _timed(torch, replay_result, reps)
    assert plan.stopped() == 0 and plan.ordinary_builds() == 0
    plan.close()
    n_mol = len(mols)
    log(f"[bench] batch: {t_tuned * 1e3:.2f} ms tuned, {t_default * 1e3:.2f} ms default cells, "
        f"{t_seq * 1e3:.1f} ms as {n_mol} sequential calls; graph replay {t_replay * 1e3:.2f} ms "
        f"({t_replay_res * 1e3:.2f} ms with the result), plan made in {plan_s:.2f} s")
    return {
        "metric": "batched molecules/s",
        "value": n_mol / t_replay,
        "unit": "molecules/s",
        "value_note": "one HIP graph replay of the recorded batch build per batch (ac_plan_launch)",
        "graph_replay_ms_per_batch": t_replay * 1e3,
        "graph_replay_with_result_ms_per_batch": t_replay_res * 1e3,
        "plan_create_s": plan_s,
        "ms_per_batch": t_tuned * 1e3,
        "ms_per_batch_default_cells": t_default * 1e3,
        "sequential_ms": t_seq * 1e3,
        "sequential_molecules_per_s": n_mol / t_seq,
        "speedup_vs_sequential": t_seq / t_tuned,
        "graph_replay_speedup_vs_sequential": t_seq / t_replay,
        "atoms": int(off[-1]),
        "counts": counts,
        "tuned_cell_mA_per_bucket": per_bucket,
        "tuner_s": tune_s,
        "config": {"workload": "512 molecules, sizes log-uniform in [500, 50000] atoms (seed 999), spheres at "
                               "0.05 atoms/A^3, vdW radii, alpha=0", "molecules": n_mol},
    }


def bench_union(acx, synth, torch, log, frames=64, reps=3):
    """Union volume and area, forward + backward, on 64 jittered frames of the
    100k-atom molecule (sigma 0.1 A, seeds 2000 + f): complexes built first,
    then V, A and their gradients timed per frame, and for all frames as one
    batch (one complex over the 64 frames, one forward, one backward)."""
    import numpy as np
    base = synth.config_100k()
    fr = [synth.jittered(base, 0.1, 2000 + f) for f in range(frames)]
    Xs = [torch.from_numpy(m.xyz).cuda() for m in fr]
    R = torch.from_numpy(base.radii).cuda()
    g = torch.ones(2, dtype=torch.float64, device="cuda")
    cs = [acx.ac_alpha_complex_device(x, R, 0.0) for x in Xs]

    def build():
        for x in Xs:
            acx.ac_alpha_complex_device(x, R, 0.0).close()

    def fwd_bwd():
        for c, x in zip(cs, Xs):
            acx.ac_union_measure_device(c, x, R)
            acx.ac_union_measure_backward(c, x, R, g)

    def fused():
        for c, x in zip(cs, Xs):
            acx.ac_union_measure_fused(c, x, R, g)

    fwd_bwd()  # first backward on a complex sorts its incidences (kept)
    fused()
    t_build = _timed(torch, build, reps) / frames
    t_fb = _timed(torch, fwd_bwd, reps) / frames
    t_fused = _timed(torch, fused, reps) / frames
    V, A = acx.ac_union_measure(cs[0], Xs[0], R)
    for c in cs:
        c.close()
    # all frames in one batch
    XB = torch.cat(Xs)
    RB = R.repeat(frames)
    off = np.arange(frames + 1, dtype=np.int64) * base.n
    cb = acx.ac_alpha_complex_batch(XB, RB, off, 0.0)
    acx.ac_union_measure_device(cb, XB, RB)
    acx.ac_union_measure_backward(cb, XB, RB, g)

    def fwd_bwd_batch():
        acx.ac_union_measure_device(cb, XB, RB)
        acx.ac_union_measure_backward(cb, XB, RB, g)

    def build_batch():
        acx.ac_alpha_complex_batch(XB, RB, off, 0.0).close()

    acx.ac_union_measure_fused(cb, XB, RB, g)
    t_fb_batch = _timed(torch, fwd_bwd_batch, reps) / frames
    t_fused_batch = _timed(torch, lambda: acx.ac_union_measure_fused(cb, XB, RB, g), reps) / frames
    t_build_batch = _timed(torch, build_batch, reps) / frames
    cb.close()
    log(f"[bench] union: per frame build {t_build * 1e3:.3f} ms, V+A fwd+bwd {t_fb * 1e3:.3f} ms "
        f"(fused {t_fused * 1e3:.3f}); batched over {frames} frames: build {t_build_batch * 1e3:.3f} ms, "
        f"fwd+bwd {t_fb_batch * 1e3:.3f} ms (fused {t_fused_batch * 1e3:.3f}) per frame")
    return {
        "metric": "V+A fwd+bwd ms",
        "value": t_fb * 1e3,
        "unit": "ms per frame",
        "higher_is_better": False,
        "build_ms_per_frame": t_build * 1e3,
        "batched_fwd_bwd_ms_per_frame": t_fb_batch * 1e3,
        "fused_fwd_bwd_ms_per_frame": t_fused * 1e3,
        "batched_fused_fwd_bwd_ms_per_frame": t_fused_batch * 1e3,
        "batched_build_ms_per_frame": t_build_batch * 1e3,
        "frame0": {"V_A3": V, "A_A2": A},
        "config": {"workload": "64 frames of the 100k-atom molecule (sphere R 78.2 A), Gaussian jitter 0.1 A, vdW "
                               "radii, alpha=0", "frames": frames, "atoms": base.n},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--alpha", type=float, default=0.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=600_000, help="atoms of the oracle's sample")
    ap.add_argument("--cache-dir", default=os.environ.get("ALPHACX_INPUT_CACHE", ""),
                    help="keep the generated input here between runs")
    ap.add_argument("--no-extras", action="store_true", help="skip the batch and union-measure workloads")
    ap.add_argument("--no-host-to-host", action="store_true", help="skip the host-array build timing")
    ap.add_argument("--no-recorded", action="store_true", help="skip the recorded-build (graph replay) timing")
    ap.add_argument("--no-tune", action="store_true", help="default cell side instead of the autotuned one")
    ap.add_argument("--cell-mA", type=int, default=0, help="fixed cell side in mA (skips the autotuner)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain device copy of 1 GiB (counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the split over several GPUs "
              "is a design, not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_1908_05944_amd as acx

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: 3 copies of {src.numel() * 4} bytes")
        del src, dst

    t0 = time.time()
    mol = synth.config_shell_3m(args.cache_dir or None)
    log(f"[bench] generated {mol.n} atoms in {time.time() - t0:.1f} s")
    dev = torch.device("cuda:0")
    xyz = torch.from_numpy(mol.xyz).to(dev)
    rad = torch.from_numpy(mol.radii).to(dev)
    stream = torch.cuda.current_stream(dev)

    # cell side from the autotuner (outside the timed region; it never changes
    # the result, only the time)
    cell_mA = args.cell_mA
    if not args.no_tune and cell_mA <= 0:
        t0 = time.perf_counter()
        cells, _ = acx.ac_tune_cells(xyz, rad, np.array([0, mol.n]), args.alpha)
        cell_mA = int(cells[0])
        log(f"[bench] tuner: cell side {cell_mA} mA ({time.perf_counter() - t0:.2f} s)")
    opts = {"cell_mA": cell_mA}

    for w in range(args.warmup):
        c = acx.ac_alpha_complex_device(xyz, rad, args.alpha, options=opts)
        counts = c.counts()
        c.close()
        log(f"[bench] warmup {w}: counts {counts}")

    # untimed profiled builds: HIP events between all stages (each event adds
    # a few microseconds of idle time, so the timed steps below record only
    # the two around the dominant kernel)
    stage_names = acx.stage_names()
    stage_tot = {}
    n_prof = 3
    for _ in range(n_prof):
        c = acx.ac_alpha_complex_device(xyz, rad, args.alpha, options={"profile": 1, "cell_mA": cell_mA})
        for k, v in c.stage_ms().items():
            stage_tot[k] = stage_tot.get(k, 0.0) + v
        c.close()
    stage_avg = {k: v / n_prof for k, v in stage_tot.items()}

    # one more build for counts (not timed)
    c = acx.ac_alpha_complex_device(xyz, rad, args.alpha, options=opts)
    counts = c.counts()
    cand = [c.candidate_count(d) for d in range(4)]
    fallbacks = c.exact_fallbacks()
    work = [c.work_count(0), c.work_count(1)]
    c.close()

    # Algorithmic work of the build (bytes and float64 operations) from the
    # measured counts; the dominant kernel is, among the stages that hold
    # exactly one kernel launch, the one with the largest event time.
    n = mol.n
    E, T, Q = cand[1], cand[2], cand[3]
    Nn = work[1]
    Pe, C = neighbour_pairs_tested(mol.X_mA, mol.R_mA.astype(np.int64) ** 2, int(round(args.alpha * 1e6)), cell_mA)
    if C != work[0]:
        log(f"[bench] host grid replication gave {C} cells, the build {work[0]}")
    B_build, F_build, alg_bytes, alg_flops = algorithmic_work(n, work[0], E, T, Q, counts, Nn, Pe)
    single = {k: v for k, v in stage_avg.items() if k in alg_bytes and v > 0}
    dom = max(single, key=lambda k: single[k])

    # timed region: exactly K steps; HIP events around the dominant kernel only
    timed = {"profile": 2 + stage_names.index(dom), "cell_mA": cell_mA}
    dom_tot = 0.0
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        c = acx.ac_alpha_complex_device(xyz, rad, args.alpha, options=timed)
        dom_tot += c.stage_ms()[dom]
        c.close()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1e3 / args.steps
    value = mol.n * args.steps / elapsed
    dom_ms = dom_tot / args.steps
    log(f"[bench] {ms_per_step:.3f} ms/step; {dom} {dom_ms:.3f} ms per launch (timed steps); untimed stages (ms): "
        + ", ".join(f"{k}={v:.3f}" for k, v in stage_avg.items()))
    # the dominant kernel: bound by what its counters show (vector issue when
    # its instruction rate is the nearer limit, else HBM), else by the larger
    # of its algorithmic times
    t_dom = dom_ms * 1e-3
    b_dom, f_dom = alg_bytes[dom], alg_flops.get(dom, 0)
    traffic = measured_traffic(dom)
    lane_ops = measured_valu_lane_ops(dom)
    issue = None if lane_ops is None else lane_ops / t_dom / (VALU_ISSUE_PEAK_T * 1e12)
    hbm_meas = None if traffic is None else traffic / t_dom / (HBM_PEAK_GBS * 1e9)
    if issue is not None and hbm_meas is not None:
        bound = "alu" if issue > hbm_meas else "hbm"
        bound_from = f"counters: vector issue {issue:.2f} of its limit, HBM traffic {hbm_meas:.2f} of peak"
    else:
        bound = "alu" if f_dom / (FP64_VECTOR_PEAK_TFLOPS * 1e12) > b_dom / (HBM_PEAK_GBS * 1e9) else "hbm"
        bound_from = "larger algorithmic time (no counters for these kernel sources)"
    hbm_view = {"achieved": b_dom / t_dom / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": b_dom / t_dom / (HBM_PEAK_GBS * 1e9), "algorithmic_bytes": b_dom}
    fp64_view = {"achieved": f_dom / t_dom / 1e12, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                 "frac": f_dom / t_dom / (FP64_VECTOR_PEAK_TFLOPS * 1e12), "algorithmic_flops": f_dom}
    # vector issue: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-operations/s
    valu_view = None if lane_ops is None else {
        "achieved": lane_ops / t_dom / 1e12, "peak": VALU_ISSUE_PEAK_T, "unit": "Tlane-op/s",
        "frac": issue, "lane_ops_per_launch": lane_ops}
    main_view = hbm_view if bound != "alu" else (valu_view if valu_view is not None else fp64_view)
    roofline = {
        "kernel": KERNEL_OF_STAGE.get(dom, dom),
        "bound": bound,
        "bound_from": bound_from,
        "achieved": main_view["achieved"],
        "peak": main_view["peak"],
        "unit": main_view["unit"],
        "frac": main_view["frac"],
        "traffic": traffic,
        "ms_per_launch": dom_ms,
        "hbm_view": hbm_view,
        "fp64_view": fp64_view,
        "valu_view": valu_view,
    }
    # the whole build: max(B / HBM peak, F / float64 peak) over the step time
    t_step = ms_per_step * 1e-3
    t_b, t_f = B_build / (HBM_PEAK_GBS * 1e9), F_build / (FP64_VECTOR_PEAK_TFLOPS * 1e12)
    tr_build = measured_traffic_total()
    build_roofline = {
        "bound": "hbm" if t_b >= t_f else "fp64",
        "frac": max(t_b, t_f) / t_step,
        "hbm_frac": t_b / t_step,
        "fp64_frac": t_f / t_step,
        "algorithmic_bytes": B_build,
        "algorithmic_flops": F_build,
        "achieved_GBs": B_build / t_step / 1e9,
        "traffic_bytes": tr_build,
        "traffic_GBs": None if tr_build is None else tr_build / t_step / 1e9,
        "pairs_tested": Pe,
        "note": "B and F from the measured counts of this build; examined triples and quadruples are "
                "counted as the candidates (a lower bound of F)",
    }
    log(f"[bench] build roofline: B {B_build / 1e6:.1f} MB, F {F_build / 1e9:.2f} GFLOP, "
        f"frac {build_roofline['frac']:.3f} ({build_roofline['bound']}); dominant {roofline['kernel']} "
        f"{roofline['frac']:.3f} ({bound})")

    # the same build as a recorded build: the pipeline captured once in a HIP
    # graph (sizes from one ordinary build, with headroom), each step one
    # graph replay over the same device-resident input; and replay + result
    # (counts read back, rows copied into a new result)
    recorded = None
    if not args.no_recorded:
        plan = acx.Plan(xyz, rad, np.array([0, n]), args.alpha, options=opts)
        plan.launch()
        plan.result().close()
        t_rep = _timed(torch, plan.launch, args.steps)

        def rep_res():
            plan.launch()
            plan.result().close()

        t_rep_res = _timed(torch, rep_res, args.steps)
        assert plan.stopped() == 0
        plan.close()
        recorded = {"ms_per_replay": t_rep * 1e3, "atoms_per_s": n / t_rep, "ms_with_result": t_rep_res * 1e3,
                    "note": "ac_plan_launch: one HIP graph replay of the whole pipeline (no host synchronisation); "
                            "with_result adds ac_plan_result (counters read back, rows copied into a new result)"}
        log(f"[bench] recorded build: {t_rep * 1e3:.3f} ms per replay, {t_rep_res * 1e3:.3f} ms with the result")

    # host-to-host: host arrays in, every result array back on the host (what
    # the paper's totals include)
    h2h = None
    if not args.no_host_to_host:
        acx.ac_alpha_complex(mol.xyz, mol.radii, args.alpha, options=opts).close()
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            acx.ac_alpha_complex(mol.xyz, mol.radii, args.alpha, options=opts).close()
            ts.append(time.perf_counter() - t0)
        h2h = {"ms": float(np.median(ts)) * 1e3, "atoms_per_s": n / float(np.median(ts)),
               "note": "ac_alpha_complex from host arrays: inputs copied up, every result array copied back "
                       "(pageable host memory), median of 3"}
        log(f"[bench] host-to-host: {h2h['ms']:.2f} ms per build")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        # bounded sample of the same workload: the atoms of a slab x <= x0
        # holding about --cpu-sample atoms, input order kept
        xs = np.sort(mol.X_mA[:, 0])
        x0 = xs[min(args.cpu_sample, n) - 1]
        sel = np.nonzero(mol.X_mA[:, 0] <= x0)[0]
        t1 = time.perf_counter()
        oc = oracle.alpha_complex(mol.xyz[sel], mol.radii[sel], args.alpha)
        dt = time.perf_counter() - t1
        cpu = {"value": len(sel) / dt, "unit": "atoms/s", "cores": 1, "kind": "oracle",
               "sample": f"{len(sel)} atoms of the 3M shell (slab x <= {x0 / 1000:.1f} A), {dt:.1f} s single-threaded",
               **host_cpu()}
        log(f"[bench] oracle sample: {len(sel)} atoms in {dt:.2f} s, counts {oc.counts()}")
        # the oracle on the small configs: 1 warm-up + 3 runs, median
        small = {}
        for name, m in (("1k", synth.config_small()), ("100k_vdw", synth.config_100k()),
                        ("100k_sas", synth.config_100k(sas=True))):
            ts = []
            for rep in range(4):
                t1 = time.perf_counter()
                oracle.alpha_complex(m.xyz, m.radii, 0.0)
                if rep:
                    ts.append(time.perf_counter() - t1)
            small[name] = {"atoms": m.n, "ms": float(np.median(ts)) * 1e3, "atoms_per_s": m.n / float(np.median(ts))}
        cpu["oracle_small_configs"] = small
        log("[bench] oracle: " + ", ".join(f"{k} {v['ms']:.1f} ms" for k, v in small.items()))

    extras = {}
    if not args.no_extras:
        extras["cell_order"] = bench_cell_order(acx, torch, log, xyz, rad, opts)
        extras["alpha_sweep"] = bench_sweep(acx, torch, log, xyz, rad, opts)
        extras["partitioned"] = bench_partition(acx, torch, log, xyz, rad, opts, mol.xyz, mol.radii)
        del xyz, rad
        torch.cuda.empty_cache()
        extras["batch"] = bench_batch(acx, synth, torch, log)
        extras["union_measure"] = bench_union(acx, synth, torch, log)
        extras["table2_split"] = bench_table2(acx, synth, torch, log)

    out = {
        "metric": "alpha-complex atoms/s at 3M atoms",
        "value": value,
        "unit": "atoms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64+f64",
        "data": "synthetic",
        "config": {"workload": "3M-atom spherical shell (R_out 279.36 A, R_in 0.7 R_out), 0.05 atoms/A^3, "
                               "vdW radii, alpha=0", "atoms": n, "alpha": args.alpha, "cell_mA": cell_mA,
                   "parallelism": "single GPU"},
        "counts": counts,
        "candidates": cand,
        "exact_fallbacks": fallbacks,
        "simplices_per_s": sum(counts) * args.steps / elapsed,
        "stage_ms": stage_avg,
        "stage_ms_note": "device time per stage, HIP events between all stages, mean of 3 untimed builds",
        "roofline": roofline,
        "build_roofline": build_roofline,
        "host_to_host": h2h,
        "recorded_build": recorded,
        "cpu_baseline": cpu,
        **extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
