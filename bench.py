#!/usr/bin/env python3
"""Throughput of the epsilon self-join on one MI355X.

One step = the whole hot path for every join of the workload: build the grid
index (bounding box, cell ids, sort, cell tables, masks, cell-ordered copy),
count pass (adjacent-cell search and refine), fill pass and row sorts, with
the sorted (i, j) pairs written to a device buffer. Inputs are resident in
HBM before the timed region starts; the output stays in HBM.

Default workload (the largest single-GPU configuration): 10,000,000 points
uniform in [0,100]^d for d = 3, 4, 5, 6 (the paper's synthetic sets, Section
VI-A), each at the eps giving a mean of 32 and of 256 neighbours per point
(calibrated by the oracle, tests/golden/eps_calibration.json): eight joins
per step, 2.9e8 .. 2.6e9 pairs each, unicomp on, binary64. Prints ONE JSON
line on stdout; everything else goes to stderr.

Beside `value` (pairs/s of the timed steps) the line carries:
  roofline         the modelled kernel with the largest time in one untimed,
                   fully profiled step; in the timed steps only its launches
                   carry HIP events. Its bound is the larger of two lower
                   bounds: HBM (algorithmic bytes at 8 TB/s) and FP64 VALU
                   (algorithmic operations, (3d - 1) per distance
                   evaluation, at 3.93e13 non-fused operations/s);
                   `traffic` is the counted HBM traffic from the summary
                   under profiles/ while the kernel's sources are unchanged;
  valu_roofline / hbm_roofline   both fractions for that kernel;
  legs             the other configurations and modes:
                     unicomp_off      the same step without unicomp;
                     fp32_band        the same step with the FP32 pre-test
                                      and FP64 band re-decision;
                     batched          the same joins delivered in 2^27-pair
                                      batches (result larger than one batch);
                     clustered_5M     5,000,000 clustered points in 2-D and
                                      3-D, FP32 pre-test + FP64 band vs FP64;
                     uniform2d_2M     2,000,000 uniform 2-D points, five eps;
                     uniform2d_10k    10,000 uniform 2-D points, eps 1;
                     brute_force      the all-pairs kernel vs the grid join;
                     rs_join          the two-set join;
                     dbscan           clustering over the CSR neighbour table;
                     serving          a Poisson request stream (p50/p99);
  cpu_baseline     the brute-force oracle on a sample of query rows, on all
                   host threads; cpu_baseline_1core the same on one thread;
  cpu_grid_baseline  the host-core grid join on whole joins of the workload.

  python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-legs] [--legs A,B]
                  [--no-cpu-baseline] [--no-serve]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP64 vector operations that are not fused multiply-adds (the pair test has
# none): 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz. Unpacked FP32
# issues at the same rate on gfx950.
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9
CALIB = os.path.join(ROOT, "tests", "golden", "eps_calibration.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workloads():
    with open(CALIB) as f:
        cal = json.load(f)
    u, c = cal["uniform_n10M"], cal["clustered_n5M"]
    return {
        "uniform_n10M_d3-6_k32-256": [
            dict(kind="uniform", n=u[k]["n"], d=u[k]["d"], seed=u[k]["seed"], eps=u[k]["eps"], tag=k)
            for k in ("d3_k32", "d3_k256", "d4_k32", "d4_k256", "d5_k32", "d5_k256", "d6_k32", "d6_k256")],
        "clustered_n5M_d2-3_median50": [
            dict(kind="clustered", n=c[k]["n"], d=c[k]["d"], seed=c[k]["seed"], eps=c[k]["eps"], tag=k)
            for k in ("d2", "d3")],
        "uniform2d_n2M_eps_sweep": [dict(kind="uniform", n=2_000_000, d=2, seed=2, eps=e, tag=f"eps{e}")
                                    for e in (0.04, 0.08, 0.12, 0.16, 0.2)],
        "uniform2d_n10k_eps1": [dict(kind="uniform", n=10_000, d=2, seed=1, eps=1.0, tag="eps1")],
    }


DEFAULT_WORKLOAD = "uniform_n10M_d3-6_k32-256"


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(workloads()))
    ap.add_argument("--unicomp", type=int, default=1)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32_band"])
    ap.add_argument("--no-legs", action="store_true", help="only the headline workload")
    ap.add_argument("--legs", default="all",
                    help="comma-separated legs to run (unicomp_off, fp32_band, batched, clustered_5M, "
                         "uniform2d_2M, uniform2d_10k, brute_force, rs_join, serving); default all")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of each host baseline sample")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving stream")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy three times (reference kernel "
                         "of known traffic for hardware byte counters)")
    return ap.parse_args()


# ------------------------------------------------------------ workloads
class Workload:
    """Device-resident points of every join of a workload and the joins'
    sizes (from an untimed count pass)."""

    def __init__(self, name, joins, torch):
        from paper_1803_04120_amd import datagen
        self.name, self.joins, self.torch = name, joins, torch
        self.points = {}
        for j in joins:
            key = (j["kind"], j["n"], j["d"], j["seed"])
            if key not in self.points:
                pts = datagen.make(j["kind"], j["n"], j["d"], j["seed"])
                self.points[key] = (pts, torch.from_numpy(pts).to("cuda"))
        self.info = None

    def x(self, j):
        return self.points[(j["kind"], j["n"], j["d"], j["seed"])][1]

    def host(self, j):
        return self.points[(j["kind"], j["n"], j["d"], j["seed"])][0]

    def size(self, sj, unicomp=True, precision="fp64"):
        info = []
        for j in self.joins:
            with sj.Index(self.x(j), j["eps"]) as ix:
                P = ix.count(unicomp=unicomp, precision=precision)
                st = ix.stats()
                off = ix.export(sj._lib.SJ_EXPORT_ROW_OFFSETS)
            lens = np.diff(off.astype(np.int64))
            info.append(dict(tag=j["tag"], n=j["n"], d=j["d"], eps=j["eps"], pairs=P, cells=st["cells"],
                             evals=st["evals"], band_rechecks=st["band_rechecks"],
                             hit_bit_bytes=st["hit_bit_bytes"], precision_used=st["precision_used"],
                             max_cell=st["max_cell_points"], max_row=st["max_row_pairs"],
                             unicomp=unicomp, row_classes=row_classes(lens)))
        self.info = info
        return info

    def max_pairs(self):
        return max(i["pairs"] for i in self.info)

    def step(self, sj, out, unicomp=True, precision="fp64"):
        total, flags = 0, []
        for j in self.joins:
            with sj.Index(self.x(j), j["eps"]) as ix:
                total += ix.count(unicomp=unicomp, precision=precision)
                ix.fill(out)
                flags.append(ix.stats()["fill_unicomp"])
        self._last_fill_unicomp = flags  # which fill kernel each join ran
        return total


def row_classes(lens):
    """Pairs in rows of each row-sort size class."""
    out = {}
    for name, lo, hi in (("le32", 0, 32), ("33_64", 33, 64), ("65_1024", 65, 1024), ("1025_8192", 1025, 8192),
                         ("gt8192", 8193, 1 << 62)):
        m = (lens >= lo) & (lens <= hi)
        out[name] = int(lens[m].sum())
    return out


# ------------------------------------------------------------ kernel models
def kernel_model(name, i):
    """(algorithmic HBM bytes, algorithmic FP64 operations) of one launch of
    kernel `name` in join i (sizes from the count pass), or None when the
    kernel is not modelled. Bytes count each array the kernel must touch
    once; operations count (3d - 1) per distance evaluation (d subtractions,
    d multiplications, d - 1 additions). With hit bits (5-D and up) the
    count pass performs every evaluation once and writes the bits, and the
    fill pass performs none: it reads the bits and writes the pairs."""
    n, d, P, cells = i["n"], i["d"], i["pairs"], i["cells"]
    U = i["evals"] if i["unicomp"] else (i["evals"] + n) // 2  # unicomp evaluations (U = (T + n) / 2)
    T = 2 * U - n
    ops_per_eval = 3 * d - 1
    bits = i.get("hit_bit_bytes", 0)
    if name.startswith("tiled_count"):
        ev = U if "unicomp" in name else T
        return n * (8 * d + 4 + 4) + 8 * (cells + 1) + bits, ev * ops_per_eval
    if name.startswith("tiled_fill_sort"):
        # coordinates, cell coordinate, cell-order and final row offsets,
        # permutation entry per point; one 8-byte (i, j) pair per result pair
        extra = 4 * d * n if name.endswith("fp32band") else 0
        return n * (8 * d + 4 + 8 + 4 + 8) + extra + 8 * P, T * ops_per_eval
    if name.startswith("tiled_fill"):
        ev = U if "unicomp" in name else T
        extra = 4 * d * n if name.endswith("fp32band") else 0
        if bits:
            return n * (4 + 8 + 4) + bits + 4 * P, 0
        return n * (8 * d + 4 + 8 + 4) + extra + 4 * P, ev * ops_per_eval
    rc = i["row_classes"]
    if name == "rowsort_wave":
        p = rc["65_1024"]
        return 8 * n + 12 * p, 0
    if name == "rowsort_block":
        return 12 * rc["1025_8192"], 0
    if name == "rowsort_group16":
        return 12 * rc["33_64"], 0
    if name == "rowsort_lane":
        return 8 * (n + 1) + 12 * rc["le32"], 0
    return None


def modelled(prof, info, fill_unicomp_flags):
    """{kernel: (launches, ms, bytes, ops)} summed over the joins of a step."""
    out = {}
    for name, (cnt, ms) in prof.items():
        b = o = 0
        ok = False
        for k, i in enumerate(info):
            m = kernel_model(name, i)
            if m is None:
                break
            ok = True
            # a join contributes only if it launched this kernel
            if launched_in(name, i, fill_unicomp_flags[k] if k < len(fill_unicomp_flags) else 0):
                b += m[0]
                o += m[1]
        if ok and (b or o):
            out[name] = (cnt, ms, b, o)
    return out


def launched_in(name, i, fill_unicomp):
    """Whether join i launches kernel `name` (which fill and row sorts run)."""
    d = i["d"]
    fused = d <= 3 and not fill_unicomp
    # an FP32 pre-test request runs the FP64 kernels where the library
    # chose them (from 6-D on)
    if name.startswith("tiled_") and name.endswith(("fp64", "fp32band")):
        if name.endswith("fp32band") != (i.get("precision_used", 0) == 1):
            return False
    if name.startswith("tiled_count"):
        return ("unicomp" in name) == bool(i["unicomp"])
    if name.startswith("tiled_fill_sort"):
        return fused
    if name.startswith("tiled_fill"):
        return (not fused) and (("unicomp" in name) == bool(fill_unicomp))
    rc = i["row_classes"]
    if name == "rowsort_wave":
        return rc["65_1024"] > 0
    if name == "rowsort_block":
        return rc["1025_8192"] > 0
    if name in ("rowsort_group16", "rowsort_lane"):
        return not fused
    return False


def roofline_of(name, cnt, ms, byts, ops):
    t = ms * 1e-3
    gbs = byts / t / 1e9
    opss = ops / t
    hbm = {"achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}
    valu = {"achieved": round(opss / 1e12, 3), "peak": round(VALU_PEAK_OPS / 1e12, 3), "unit": "TFLOP/s",
            "frac": round(opss / VALU_PEAK_OPS, 4)}
    bound = "alu" if ops / VALU_PEAK_OPS > byts / (HBM_PEAK_GBS * 1e9) else "hbm"
    main = valu if bound == "alu" else hbm
    return dict(bound=bound, kernel=name, achieved=main["achieved"], peak=main["peak"], unit=main["unit"],
                frac=main["frac"], avg_launch_us=round(1e3 * ms / cnt, 3), launches=cnt,
                bytes_per_launch=int(byts / cnt), ops_per_launch=int(ops / cnt)), hbm, valu


# Sources compiled into each family of modelled kernels: a traffic figure
# measured with hardware counters is only reported while these are unchanged.
KERNEL_SOURCES = {
    "tiled_": ["k_tile.hip", "sj_device.h", "sj_args.h"],
    "join_": ["k_join.hip", "sj_device.h", "sj_args.h"],
    "rowsort_": ["k_rowsort.hip", "sj_device.h", "sj_args.h"],
    "brute_": ["k_brute.hip", "sj_device.h", "sj_args.h"],
    "rs_": ["k_rs.hip", "sj_device.h", "sj_args.h"],
}


def kernel_source_hash(name):
    import hashlib
    for prefix, files in KERNEL_SOURCES.items():
        if name.startswith(prefix):
            h = hashlib.sha256()
            for f in files:
                with open(os.path.join(ROOT, "paper_1803_04120_amd", "csrc", f), "rb") as fh:
                    h.update(fh.read())
            return h.hexdigest()[:16]
    return None


def measured_traffic(name, workload):
    """HBM bytes per launch of `name` on `workload` from the counter summary
    under profiles/ (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when
    there is none or the kernel's sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{name}_{workload}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("source_sha256_16") != kernel_source_hash(name):
        return None
    try:
        return int(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def pipeline_bytes(n, d, cells, pairs):
    """Algorithmic bytes of the whole path for one join: read the input,
    write and read the cell-ordered copy (24 n d), the point map (4 n), the
    cell tables written and read (32 |G|) and each pair written once (8 P)."""
    return 24 * n * d + 4 * n + 32 * cells + 8 * pairs


# ------------------------------------------------------------ timing helpers
def timed_steps(fn, steps, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot = 0
    for _ in range(steps):
        tot += fn()
    torch.cuda.synchronize()
    return tot, time.perf_counter() - t0


def profiled_step(fn, _lib, torch, select=""):
    _lib.profile_select(select)
    _lib.profile_enable(True)
    fn()
    torch.cuda.synchronize()
    _lib.profile_enable(False)
    _lib.profile_select("")
    return _lib.profile_read()


def sweep_leg(sj, _lib, torch, wl, steps, unicomp=True, precision="fp64", label=""):
    """Timed steps of a workload plus the roofline of its dominant kernel
    (events on that kernel's launches of a final step)."""
    info = wl.size(sj, unicomp, precision)
    out = torch.empty((wl.max_pairs(), 2), dtype=torch.int32, device="cuda")
    fn = lambda: wl.step(sj, out, unicomp, precision)  # noqa: E731
    fn()
    tot, dt = timed_steps(fn, steps, torch)
    prof = profiled_step(fn, _lib, torch)
    mod = modelled(prof, info, wl._last_fill_unicomp)
    res = {"pairs_per_s": tot / dt, "ms_per_step": 1e3 * dt / steps, "steps": steps,
           "pairs_per_step": tot // steps, "unicomp": unicomp, "precision": precision,
           "per_join": [{k: v for k, v in i.items() if k != "row_classes"} for i in info],
           "kernels_ms": {k: round(v[1], 4) for k, v in prof.items()}}
    if mod:
        dom = max(mod, key=lambda k: mod[k][1])
        r, hbm, valu = roofline_of(dom, *mod[dom])
        # the profiles are of the FP64 runs: a request for the FP32 pre-test
        # runs other launches of the same kernels
        r["traffic"] = measured_traffic(dom, wl.name) if precision == "fp64" else None
        res["roofline"] = r
        res["hbm_roofline"], res["valu_roofline"] = hbm, valu
    log(f"[bench] {label or wl.name} {precision} unicomp={unicomp}: {res['pairs_per_s']:.4g} pairs/s, "
        f"{res['ms_per_step']:.3f} ms/step" + (f", {res['roofline']['kernel']} {res['roofline']['bound']} "
                                                f"frac {res['roofline']['frac']}" if mod else ""))
    del out
    torch.cuda.empty_cache()
    return res


# ------------------------------------------------------------ host baselines
def host_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "omp_threads": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))}


def _set_omp_threads(k):
    import ctypes
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(k))
        return True
    except OSError:
        return False


def cpu_baseline(wl, target_s, threads):
    """The brute-force oracle on a bounded sample of query rows (all n
    candidates each) of every join of the workload, on `threads` host
    threads, scaled to pairs/s."""
    from oracle import reference
    _set_omp_threads(threads)
    g = np.random.default_rng(12345)
    # pilot: cost per query row of each join
    per_row = []
    for j in wl.joins:
        pts = wl.host(j)
        rows = g.choice(pts.shape[0], size=16, replace=False)
        t0 = time.perf_counter()
        reference.count_rows(pts, j["eps"], rows)
        per_row.append((time.perf_counter() - t0) / 16)
    rows_per = max(16, int(target_s / sum(per_row)))
    pairs = 0
    t0 = time.perf_counter()
    for j in wl.joins:
        pts = wl.host(j)
        rows = g.choice(pts.shape[0], size=min(rows_per, pts.shape[0]), replace=False)
        pairs += int(reference.count_rows(pts, j["eps"], rows).sum())
    dt = time.perf_counter() - t0
    _set_omp_threads(host_info()["omp_threads"])
    return {"value": pairs / dt, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"{rows_per} random query rows x all n candidates for each of the {len(wl.joins)} joins "
                      f"of {wl.name} ({pairs} pairs in {dt:.1f} s); rate = sample pairs / sample time"}


def cpu_grid_baseline(wl, target_s, threads):
    """The host-core grid join (oracle/cpu_grid_join.c: the same grid method,
    count then sorted fill) on whole joins of the workload, in order, until
    about target_s seconds have passed."""
    from oracle import reference
    pairs, done = 0, []
    t0 = time.perf_counter()
    for j in wl.joins:
        counts, out = reference.grid_join(wl.host(j), j["eps"])
        pairs += out.shape[0]
        done.append(j["tag"])
        del out
        if time.perf_counter() - t0 > target_s:
            break
    dt = time.perf_counter() - t0
    return {"value": pairs / dt, "unit": "pairs/s", "cores": threads, "kind": "cpu_grid_join",
            "sample": f"whole joins {done} of {wl.name} with sorted (i,j) output ({pairs} pairs in {dt:.1f} s)"}


# ------------------------------------------------------------ other legs
def batched_leg(sj, torch, wl, cap):
    """The workload's joins delivered as runs of at most cap pairs (at least
    3), each handed to a callback in device memory; one warm pass, one timed."""
    def one_pass():
        nb, tot = [], 0
        for j in wl.joins:
            with sj.Index(wl.x(j), j["eps"]) as ix:
                bl = []
                tot += ix.batches(lambda p, np_, b, r0, r1: bl.append(np_), unicomp=True, precision="fp64",
                                  batch_capacity_pairs=cap, min_batches=3)
                nb.append(len(bl))
        return nb, tot
    one_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nb, tot = one_pass()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"[bench] batched ({cap} pairs): {tot / dt:.4g} pairs/s, batches {nb}")
    return {"capacity_pairs": cap, "min_batches": 3, "batches_per_join": nb, "pairs_per_s": tot / dt,
            "ms_per_step": 1e3 * dt, "note": "one warm pass then one timed pass; every run delivered in device memory to a callback"}


def brute_leg(sj, _lib, torch):
    """The all-pairs kernel beside the grid join on the same inputs: the
    10,000-point 2-D workload and a 6-D set whose grid degenerates."""
    from paper_1803_04120_amd import datagen
    res = []
    for (n, d, eps, seed) in ((10_000, 2, 1.0, 1), (200_000, 6, 100.0 / 3.0, 61)):
        x = torch.from_numpy(datagen.uniform(n, d, seed)).cuda()
        P = sj.bruteforce(x, eps).shape[0]
        out = torch.empty((P, 2), dtype=torch.int32, device="cuda")
        sj.bruteforce(x, eps, out=out)
        reps = 3 if n > 50_000 else 20
        _, dt = timed_steps(lambda: sj.bruteforce(x, eps, out=out).shape[0], reps, torch)
        prof = profiled_step(lambda: sj.bruteforce(x, eps, out=out), _lib, torch)
        ms_k = sum(v[1] for k, v in prof.items() if k.startswith("brute_"))
        ops = 2 * n * n * (3 * d - 1)  # count and fill passes
        _, gdt = timed_steps(lambda: sj.selfjoin(x, eps).shape[0], reps, torch)
        res.append({"n": n, "d": d, "eps": eps, "pairs": P, "brute_ms": 1e3 * dt / reps,
                    "brute_pairs_per_s": P * reps / dt, "grid_ms": 1e3 * gdt / reps,
                    "grid_pairs_per_s": P * reps / gdt,
                    "roofline": {"bound": "alu", "kernel": "brute_count+brute_fill",
                                 "achieved": round(ops / (ms_k * 1e-3) / 1e12, 3),
                                 "peak": round(VALU_PEAK_OPS / 1e12, 3), "unit": "TFLOP/s",
                                 "frac": round(ops / (ms_k * 1e-3) / VALU_PEAK_OPS, 4)}})
        log(f"[bench] brute force n={n} d={d}: {1e3 * dt / reps:.3f} ms vs grid {1e3 * gdt / reps:.3f} ms")
        del out, x
    torch.cuda.empty_cache()
    return res


def rs_model(name, nq, ns, d, P, evals):
    """(algorithmic HBM bytes, FP64 operations) of one two-set join launch:
    every query's coordinates, sub-cell, row id and row offsets once, S's
    coordinates, sub-cell and id once, the result once; (3d - 1) operations
    per distance evaluation."""
    ops = evals * (3 * d - 1)
    if name.startswith("tiled_count"):
        return nq * (8 * d + 4 + 4 + 4) + ns * (8 * d + 4), ops
    if name.startswith("tiled_fill_sort"):
        return nq * (8 * d + 4 + 4 + 8 + 8) + ns * (8 * d + 4 + 4) + 8 * P, ops
    if name.startswith("tiled_fill"):
        return nq * (8 * d + 4 + 4 + 8) + ns * (8 * d + 4 + 4) + 4 * P, ops
    return None


def rs_leg(sj, _lib, torch):
    """R x S on the tiled kernel: 10^6 uniform 2-D queries against the 2M
    indexed points, five eps; timed calls, then one profiled call per eps
    for the count and fill kernels' rooflines."""
    from paper_1803_04120_amd import datagen
    S = torch.from_numpy(datagen.uniform(2_000_000, 2, 2)).cuda()
    R = torch.from_numpy(datagen.uniform(1_000_000, 2, 1002)).cuda()
    out = torch.empty((26_000_000, 2), dtype=torch.int32, device="cuda")
    per, kern = [], {}
    for e in (0.04, 0.08, 0.12, 0.16, 0.2):
        with sj.Index(S, e) as ix:
            ix.join_rs(R, out=out)
            st = _lib.last_run_stats()
            reps = 3
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                got = ix.join_rs(R, out=out)
            torch.cuda.synchronize()
            per.append((e, int(got.shape[0]), (time.perf_counter() - t0) / reps, int(st["evals"])))
            _lib.profile_select("")
            _lib.profile_enable(True)
            ix.join_rs(R, out=out)
            torch.cuda.synchronize()
            _lib.profile_enable(False)
            for name, (cnt, ms) in _lib.profile_read().items():
                m = rs_model(name, 1_000_000, 2_000_000, 2, int(got.shape[0]), int(st["evals"]))
                if m is None:
                    continue
                k = kern.setdefault(name, [0, 0.0, 0, 0])
                k[0] += cnt
                k[1] += ms
                k[2] += m[0]
                k[3] += m[1]
    tp, tt = sum(p for _, p, _, _ in per), sum(t for _, _, t, _ in per)
    log(f"[bench] two-set join: {tp / tt:.4g} pairs/s")
    roof = {}
    for name, (cnt, ms, b, o) in kern.items():
        r, hbm, valu = roofline_of(name, cnt, ms, b, o)
        r["hbm_frac"], r["valu_frac"] = hbm["frac"], valu["frac"]
        r["traffic"] = measured_traffic(name, "uniform2d_q1M_s2M_eps_sweep")
        roof[name] = r
    return {"queries": 1_000_000, "indexed": 2_000_000, "pairs_per_s": tp / tt, "ms_per_sweep": 1e3 * tt,
            "per_eps": [{"eps": e, "pairs": p, "ms": round(1e3 * t, 3), "evals": ev} for e, p, t, ev in per],
            "roofline": roof,
            "note": "count + fill + row sort per call (sj_join_rs, grid-row tiled kernel), index on the 2M "
                    "uniform 2-D points"}


def dbscan_leg(sj, torch, wl):
    res = []
    for j in wl.joins:
        x = wl.x(j)
        sj.dbscan(x, j["eps"], 50)
        reps = 3
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            labels, nc = sj.dbscan(x, j["eps"], 50)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        noise = int((labels == -1).sum().item())
        res.append({"join": j["tag"], "n": j["n"], "eps": j["eps"], "min_pts": 50, "ms": round(1e3 * dt, 3),
                    "clusters": nc, "noise_points": noise, "points_per_s": j["n"] / dt})
        log(f"[bench] dbscan {j['tag']}: {1e3 * dt:.2f} ms, {nc} clusters")
    return res


def calibrate_eps_gpu(sj, x, k, eps0):
    """eps whose mean neighbour count (self excluded) is about k, by bisection
    on the GPU count pass (a few builds of the request's own points)."""
    n = x.shape[0]
    lo, hi = eps0 * 0.05, eps0 * 2.0

    def mean_k(e):
        with sj.Index(x, e) as ix:
            return ix.count(unicomp=True) / n - 1.0
    for _ in range(14):
        mid = (lo * hi) ** 0.5
        if mean_k(mid) < k:
            lo = mid
        else:
            hi = mid
    return (lo * hi) ** 0.5


def serving_leg(args, sj, torch):
    """Poisson stream of self-join requests through the continuous-batching
    server: n log-uniform in [1e3, 2e6], d uniform in 2..6, uniform or
    clustered points, eps for a target mean neighbour count log-uniform in
    [4, 128], FP32 pre-test path. A closed-loop pass (all requests at once)
    gives the saturation rate; open-loop passes run at 0.7 and 0.5 of it.
    The same requests run one at a time on the plain FP64 path give the
    reference rate."""
    from paper_1803_04120_amd import datagen
    from paper_1803_04120_amd.serve import Server, run_stream, uniform_eps_for_k
    descs = datagen.serving_requests(args.serve_requests, seed=5)
    reqs = []
    t0 = time.perf_counter()
    for q in descs:
        pts = datagen.make(q["kind"], q["n"], q["d"], q["seed"])
        x = torch.from_numpy(pts).cuda()
        eps = uniform_eps_for_k(q["n"], q["d"], q["k"])
        if q["kind"] == "clustered":
            eps = calibrate_eps_gpu(sj, x, q["k"], eps)
        reqs.append({"points": x, "eps": eps, "precision": "fp32_band", "unicomp": True,
                     "expected_pairs": int(q["n"] * (q["k"] + 1)), "n": q["n"], "d": q["d"]})
    torch.cuda.synchronize()
    log(f"[bench] serving: {len(reqs)} requests prepared in {time.perf_counter() - t0:.1f} s")
    # the same requests alone, plain FP64 path (and their algorithmic bytes)
    solo_pairs, alg = 0, 0
    t0 = time.perf_counter()
    for r in reqs:
        with sj.Index(r["points"], r["eps"]) as ix:
            P = ix.count(unicomp=True, precision="fp64")
            st = ix.stats()
            out = torch.empty((max(P, 1), 2), dtype=torch.int32, device="cuda")
            ix.fill(out)
            del out
        solo_pairs += P
        alg += pipeline_bytes(r["n"], r["d"], st["cells"], P)
    torch.cuda.synchronize()
    solo_dt = time.perf_counter() - t0
    # the solo pass's result tensors stay in torch's cache: hand them back so
    # the server's own allocations do not compete with them
    torch.cuda.empty_cache()
    from paper_1803_04120_amd import _lib
    free, total = torch.cuda.mem_get_info()
    log(f"[bench] serving: device free {free / 2**30:.1f} GiB, library {_lib.memory_info()}")
    budget = 64 << 30
    res = {"requests": len(reqs), "slots": args.serve_slots, "mem_budget_bytes": budget,
           "precision": "fp32_band",
           "n_range": [int(min(r["n"] for r in reqs)), int(max(r["n"] for r in reqs))],
           "solo_fp64": {"pairs_per_s": solo_pairs / solo_dt, "s": round(solo_dt, 3),
                         "hbm_frac": round(alg / solo_dt / 1e9 / HBM_PEAK_GBS, 5)}}
    with Server(slots=args.serve_slots, mem_budget_bytes=budget) as srv:
        done, span = run_stream(srv, reqs, np.zeros(len(reqs)))
        sat = len(reqs) / span
        res["saturation_req_per_s"] = round(sat, 2)
        res["closed_loop_pairs_per_s"] = sum(c["npairs"] for c in done) / span
        for frac in (0.7, 0.5):
            arr = datagen.poisson_arrivals(len(reqs), frac * sat, seed=6)
            done, span2 = run_stream(srv, reqs, arr)
            lat = np.array([c["latency_ms"] for c in done])
            pairs = sum(c["npairs"] for c in done)
            res[f"at_{frac}"] = {
                "rate_req_per_s": round(frac * sat, 2), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "p99_over_p50": round(float(np.percentile(lat, 99) / np.percentile(lat, 50)), 2),
                "mean_queue_ms": round(float(np.mean([c["queue_ms"] for c in done])), 3),
                "pairs_per_s": pairs / span2, "vs_solo_fp64": round((pairs / span2) / (solo_pairs / solo_dt), 3),
                "hbm_frac": round(alg / span2 / 1e9 / HBM_PEAK_GBS, 5),
                "errors": int(sum(c["status"] != 0 for c in done))}
            log(f"[bench] serving at {frac} x saturation: p50 {res[f'at_{frac}']['p50_ms']} ms, "
                f"p99 {res[f'at_{frac}']['p99_ms']} ms, {pairs / span2:.4g} pairs/s")
        res["over_estimate"] = srv.info()["over_estimate"]
    del reqs
    torch.cuda.empty_cache()
    return res


# ------------------------------------------------------------ main
def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the self-join path here is single-GPU)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    import paper_1803_04120_amd as sj
    from paper_1803_04120_amd import _lib

    W = workloads()
    t_start = time.perf_counter()
    wl = Workload(args.workload, W[args.workload], torch)
    log(f"[bench] workload {args.workload}: {len(wl.joins)} joins, points generated")
    uni, prec = bool(args.unicomp), args.precision
    info = wl.size(sj, uni, prec)
    for i in info:
        log(f"[bench]   {i['tag']}: n={i['n']} d={i['d']} eps={i['eps']} pairs={i['pairs']} evals={i['evals']}")
    out = torch.empty((wl.max_pairs(), 2), dtype=torch.int32, device="cuda")

    def step():
        return wl.step(sj, out, uni, prec)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # every kernel of one untimed step (for the log), which also names the
    # dominant modelled kernel: the one the timed region times with events
    all_prof = profiled_step(step, _lib, torch)
    log("[bench] all kernels of one step:")
    for k, (cnt, ms) in sorted(all_prof.items(), key=lambda kv: -kv[1][1]):
        log(f"[bench]   {k:30s} launches={cnt:6d} total={ms:9.3f} ms avg={1e3 * ms / cnt:9.2f} us")
    fill_flags = list(wl._last_fill_unicomp)
    first = modelled(all_prof, info, fill_flags)
    if not first:
        raise RuntimeError(f"no modelled kernel among {sorted(all_prof)}")
    dom = max(first, key=lambda k: first[k][1])
    # timed region: HIP events (on the launch stream) only around the
    # dominant kernel's launches of the last timed step. A timing event
    # costs the stream about 24 us of idle time (measured in the kernel
    # trace), so timing every launch of every step would slow the steps.
    _lib.profile_select(dom)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pairs_total = 0
    for k in range(args.steps):
        if k == args.steps - 1:
            _lib.profile_enable(True)
        pairs_total += step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    _lib.profile_enable(False)
    _lib.profile_select("")
    prof = _lib.profile_read()
    ms_per_step = 1e3 * dt / args.steps
    value = pairs_total / dt
    log(f"[bench] {args.steps} steps in {dt:.3f}s, {ms_per_step:.3f} ms/step, {value:.4g} pairs/s")
    mod = modelled(prof, info, fill_flags)
    if dom not in mod:
        raise RuntimeError(f"the timed region recorded no launch of {dom}")
    roofline, hbm_r, valu_r = roofline_of(dom, *mod[dom])
    roofline["traffic"] = measured_traffic(dom, args.workload)
    pipe = sum(pipeline_bytes(i["n"], i["d"], i["cells"], i["pairs"]) for i in info)
    ops_step = sum(mod_i[3] for mod_i in first.values())
    pipeline = {"alg_bytes_per_step": pipe, "achieved_GBs": round(pipe / (ms_per_step * 1e-3) / 1e9, 2),
                "frac_of_hbm_peak": round(pipe / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "alg_fp64_ops_per_step": ops_step,
                "frac_of_valu_peak": round(ops_step / (ms_per_step * 1e-3) / VALU_PEAK_OPS, 4)}
    del out
    torch.cuda.empty_cache()

    legs = {}
    chosen = None if args.legs == "all" else set(args.legs.split(","))

    def want(name):
        return chosen is None or name in chosen
    if not args.no_legs:
        if args.workload == DEFAULT_WORKLOAD:
            if want("unicomp_off"):
                legs["unicomp_off"] = sweep_leg(sj, _lib, torch, wl, 2, unicomp=False, label="unicomp off")
                legs["unicomp_off"]["vs_unicomp_on"] = round(legs["unicomp_off"]["pairs_per_s"] / value, 4)
            if want("fp32_band"):
                legs["fp32_band"] = sweep_leg(sj, _lib, torch, wl, 2, precision="fp32_band", label="fp32+band")
                legs["fp32_band"]["vs_fp64"] = round(legs["fp32_band"]["pairs_per_s"] / value, 4)
            if want("batched"):
                legs["batched"] = batched_leg(sj, torch, wl, 1 << 27)
                legs["batched"]["vs_unbatched"] = round(legs["batched"]["pairs_per_s"] / value, 4)
        for name, key, steps in (("clustered_5M", "clustered_n5M_d2-3_median50", 3),
                                 ("uniform2d_2M", "uniform2d_n2M_eps_sweep", 20),
                                 ("uniform2d_10k", "uniform2d_n10k_eps1", 50)):
            if key == args.workload or not want(name):
                continue
            w2 = Workload(key, W[key], torch)
            legs[name] = {"workload": key, "fp64": sweep_leg(sj, _lib, torch, w2, steps, label=key)}
            if name == "uniform2d_2M":
                b = batched_leg(sj, torch, w2, 1 << 24)
                b["vs_unbatched"] = round(b["pairs_per_s"] / legs[name]["fp64"]["pairs_per_s"], 4)
                legs[name]["batched"] = b
            if name == "clustered_5M":
                b = sweep_leg(sj, _lib, torch, w2, steps, precision="fp32_band", label=key)
                b["vs_fp64"] = round(b["pairs_per_s"] / legs[name]["fp64"]["pairs_per_s"], 4)
                legs[name]["fp32_band"] = b
                legs["dbscan"] = dbscan_leg(sj, torch, w2)
            if name == "uniform2d_10k" and not args.no_cpu_baseline:
                from oracle import reference
                j = w2.joins[0]
                t0 = time.perf_counter()
                P = reference.pairs(w2.host(j), j["eps"]).shape[0]
                legs[name]["cpu_oracle_full"] = {"value": P / (time.perf_counter() - t0), "unit": "pairs/s",
                                                 "cores": host_info()["omp_threads"], "kind": "oracle",
                                                 "sample": "the whole 10,000-point join"}
            del w2
            torch.cuda.empty_cache()
        if want("brute_force"):
            legs["brute_force"] = brute_leg(sj, _lib, torch)
        if want("rs_join"):
            legs["rs_join"] = rs_leg(sj, _lib, torch)
        if not args.no_serve and want("serving"):
            legs["serving"] = serving_leg(args, sj, torch)

    if args.calib_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] calibration copy: 3 x 1 GiB read + 1 GiB written")
        del src, dst

    cpu = cpu1 = cpu_grid = None
    hi = host_info()
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, args.cpu_seconds, hi["omp_threads"])
        log(f"[bench] cpu oracle baseline {cpu['value']:.4g} pairs/s on {cpu['cores']} threads")
        cpu1 = cpu_baseline(wl, args.cpu_seconds / 2, 1)
        log(f"[bench] cpu oracle baseline {cpu1['value']:.4g} pairs/s on 1 thread")
        cpu_grid = cpu_grid_baseline(wl, args.cpu_seconds, hi["omp_threads"])
        log(f"[bench] cpu grid-join baseline {cpu_grid['value']:.4g} pairs/s on {cpu_grid['cores']} threads")

    rec = {
        "metric": "self-join neighbor pairs/s",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "joins": [f"{i['tag']} (n={i['n']}, d={i['d']}, eps={i['eps']})"
                                                        for i in info],
                   "unicomp": uni, "precision": prec, "output": "sorted (i,j) pairs in HBM"},
        "roofline": roofline,
        "hbm_roofline": hbm_r,
        "valu_roofline": valu_r,
        "pipeline": pipeline,
        "cpu_baseline": cpu,
        "cpu_baseline_1core": cpu1,
        "cpu_grid_baseline": cpu_grid,
        "host": hi,
        "per_join": [{k: v for k, v in i.items() if k != "row_classes"} for i in info],
        "kernels_ms": {k: round(v[1], 4) for k, v in all_prof.items()},
        "legs": legs,
        "bench_wall_s": round(time.perf_counter() - t_start, 1),
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
