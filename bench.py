#!/usr/bin/env python3
"""Benchmark of the all-pairs energy+force pass on one MI355X.

One step = one coulomb_forces call (energy fused with forces, mixed precision:
FP32 pairs, FP64 folds) on N = 100 000 charges of the warped-lattice workload
(sigma = 0.02 h), inputs resident in HBM before the timed region.  The metric
counts ordered pair interactions, N(N-1) per call.

Printed: one JSON line with the driver's fields plus
  roofline      the symmetric pair kernel against the FP32 vector peak
                (algorithmic flops: 13 per ordered pair; kernel time from HIP
                events recorded around that kernel on its stream);
  cpu_baseline  the CPU oracle on a bounded sample of rows of the same input;
  extra         FP64 energy+forces, HVP (both precisions), energy-only rates and the
                Riesz-s generalisation (s = 2, 3 mixed; s = 2 and 1.7 FP64: powers of
                1/r when 2s is an integer, pow otherwise).

  relax         the batched subdomain relax of 256 patches (sizes U{200..5000})
                on the same configuration, mixed path, seconds per batch ("cycle");
                mixed vs plain FP64 on the first 64 of those patches with the
                per-patch energy agreement (same minimum: E_sub to 1e-12), an
                ablation (the mixed path's model with FP64 pairs only), and both
                paths from common near-minimum starts (same basin, equal E).
  defect_cycle  one defect-targeted cycle of the paper's method (Sec. II.C):
                T = 1000 zones on fresh positions of the same workload, local
                energies and defect list, zone centres and oscillating radii,
                first-fit batches of mutually apart zones, mixed relax and
                greedy commit; seconds per cycle and the energy it gains.
                --no-relax skips it with the other relax measurements.

Other modes: --cycles K runs K perturb-and-relax cycles (64 kicked patches
each, greedy commit) and prints energy versus wall time; --relax-only mixed|fp64
times one relax call on the 256 patches of workload 4; --defect-only mixed|fp64
runs one defect-targeted cycle; --border-sweep N runs one such cycle per
boundary population around Eq. 4 under the border-interior split (Sec. II.B);
--copy-probe runs a plain device copy of known size (to calibrate HBM byte
counters); --pair-scaling N1,N2,... times the mixed energy+forces call at each N.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-extra]
                       [--no-relax] [--tune] [--cycles K --cycle-n N --cycle-precision P]
                       [--relax-only mixed|fp64] [--defect-only mixed|fp64 --defect-T T
                       --defect-kappa K] [--no-defect] [--border-sweep N] [--copy-probe]
                       [--pair-scaling N1,N2,...]
"""
import argparse
import ctypes
import statistics
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_PEAK_TFLOPS = 157.3     # MI355X FP32 vector peak
# unpacked FP32 issue: one wave64 instruction per four clocks per SIMD, 3.6-3.8e13 lane
# instructions/s as timed by paper_2609_24722_amd/issue_rates, x 2 flops for an FMA
FP32_UNPACKED_FMA_TFLOPS = 76.0
FLOPS_EF = 13                # energy+forces: 2 sub, 3 r^2, 1 rsqrt, 1 add, 2 r^-3, 4 FMA
FLOPS_EF_EXEC = 17           # executed per unordered pair: the same plus the j side's two FMAs
FLOPS_HVP = 24
FLOPS_RIESZ = 15             # Riesz-s: 2 sub, 3 r^2, log2, mul, exp2, 2 energy fma, 1 mul, 4 FMA


def hip_runtime():
    import torch
    path = os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so")
    h = ctypes.CDLL(path if os.path.exists(path) else "libamdhip64.so.7")
    h.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    h.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
    h.hipEventSynchronize.argtypes = [ctypes.c_void_p]
    h.hipEventDestroy.argtypes = [ctypes.c_void_p]
    return h


def timed(fn, steps, warmup, lib, hip):
    """Run fn warmup+steps times; returns (ms per call over the region, mean
    ms of the dominant pair kernel from events recorded around it)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = []
    for _ in range(steps):
        a, b = ctypes.c_void_p(), ctypes.c_void_p()
        hip.hipEventCreate(ctypes.byref(a))
        hip.hipEventCreate(ctypes.byref(b))
        evs.append((a, b))
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    marks[0].record()
    for k, (a, b) in enumerate(evs):
        lib.coulomb_set_kernel_events(a, b)
        fn()
        marks[k + 1].record()
    torch.cuda.synchronize()
    lib.coulomb_set_kernel_events(None, None)
    region_ms = marks[0].elapsed_time(marks[-1]) / steps
    calls = [marks[k].elapsed_time(marks[k + 1]) for k in range(steps)]
    ks = []
    for a, b in evs:
        ms = ctypes.c_float()
        hip.hipEventElapsedTime(ctypes.byref(ms), a, b)
        ks.append(ms.value)
        hip.hipEventDestroy(a)
        hip.hipEventDestroy(b)
    timed.last = {"call_ms_median": statistics.median(calls), "call_ms_min": min(calls),
                  "kernel_ms_median": statistics.median(ks), "kernel_ms_min": min(ks)}
    return region_ms, sum(ks) / len(ks)


def cpu_baseline(x, y, seconds=15.0):
    """The oracle's E+F sums (every row against all N) on the same input,
    repeated over row blocks until about `seconds` of CPU work is done."""
    import numpy as np
    import oracle as O
    n = x.size
    block = np.arange(0, n, max(1, n // 2000), dtype=np.int32)  # an even spread of rows
    rows_done = 0
    t = time.perf_counter()
    k = 0
    while time.perf_counter() - t < seconds:
        O.rows(x, y, (block + k) % n)
        rows_done += block.size
        k += 1
    dt = time.perf_counter() - t
    cores = O.num_threads()
    # the same sums on one thread, over a smaller sample (about a fifth of the time)
    O.set_threads(1)
    r1 = 0
    t1 = time.perf_counter()
    k1 = 0
    while time.perf_counter() - t1 < seconds / 5:
        O.rows(x, y, (block[: max(1, block.size // 8)] + k1) % n)
        r1 += max(1, block.size // 8)
        k1 += 1
    d1 = time.perf_counter() - t1
    O.set_threads(cores)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": rows_done * (n - 1) / dt, "unit": "pair-interactions/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{rows_done} rows (blocks of {block.size} evenly spread charges) of the N={n} input, "
                      f"each against all {n - 1} others: FP64 Neumaier sums of 1/r and (r_i - r_j)/r^3, "
                      f"{dt:.1f} s on {cores} threads",
            "value_1_thread": r1 * (n - 1) / d1, "cpu_model": model}


def progress(msg):
    """A progress line on stderr (the result line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def relax_comparison(xt, yt, subset):
    """Workload 4: 256 patches, sizes U{200..5000}, centres seeded, start at the
    snapshot; gtol 1e-3 on the exact reduced gradient.

    Both paths on all 256 patches (the plain FP64 path with its default
    truncated-Newton polish), the paper's optimiser (L-BFGS, no polish) on the
    plain path for the first `subset` patches, an ablation (the mixed model
    with FP64 pairs only), and the comparison at equal energy: from the plain
    path's endpoints kicked by 0.02 h both paths relax the subset, the patches
    whose endpoints agree (E_sub to 1e-12, positions within 1e-3 h) are relaxed
    again as a batch of their own, and only that rerun -- re-checked to the
    same 1e-12 -- gives the speedup at equal E."""
    import numpy as np
    import torch
    from paper_2609_24722_amd import FP64, MIXED, workloads as W
    from paper_2609_24722_amd import relax as R
    n = xt.numel()
    h = W.spacing(n)
    centres, sizes = W.patch_draws(n, 256, 200, 5000, 1104)
    ptr, idx = R.build_patches(xt, yt, centres, sizes)
    st = lambda r: np.bincount(r.status.cpu().numpy(), minlength=4).tolist()

    def run(pp, ii, prec, sx=None, sy=None, **kw):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = R.relax_subdomains(xt, yt, pp, ii, sx, sy, precision=prec, gtol=1e-3, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        progress(f"relax {'mixed' if prec == MIXED else 'fp64'} {pp.size - 1} patches {kw or ''}: {dt:.2f} s")
        return dt, r

    def agree(pp, ra, rb):
        """per patch: relative E_sub difference and largest displacement (units of h)"""
        ea, eb = ra.e_sub.cpu().numpy(), rb.e_sub.cpu().numpy()
        xa, ya, xb, yb = (a.cpu().numpy() for a in (ra.x, ra.y, rb.x, rb.y))
        disp = np.array([np.hypot(xa[pp[p]:pp[p + 1]] - xb[pp[p]:pp[p + 1]],
                                  ya[pp[p]:pp[p + 1]] - yb[pp[p]:pp[p + 1]]).max() for p in range(pp.size - 1)])
        return np.abs(ea - eb) / np.abs(eb), disp / h

    def sub_batch(pp, ii, keep):
        """the patches `keep` of batch (pp, ii) as a batch of their own"""
        ih = ii.cpu().numpy()
        sel = np.concatenate([np.arange(pp[p], pp[p + 1]) for p in keep])
        return R.offsets(np.diff(pp)[keep]), torch.tensor(ih[sel], device=xt.device), sel

    t_all, r_all = run(ptr, idx, MIXED)
    t_all_fp, r_all_fp = run(ptr, idx, FP64)
    rel256, disp256 = agree(ptr, r_all, r_all_fp)
    same256 = (rel256 <= 1e-12) & (disp256 <= 1e-3)
    ps = ptr[:subset + 1].copy()
    ids = idx[:int(ps[-1])].contiguous()
    t_mix, r_mix = run(ps, ids, MIXED)
    t_fp, r_fp = run(ps, ids, FP64)
    t_fp_lb, r_fp_lb = run(ps, ids, FP64, polish=R.POLISH_LBFGS)
    t_abl, r_abl = run(ps, ids, MIXED, inner_tol=1e300)
    # equal energy: common near-minimum starts (the plain path's endpoints kicked by 0.02 h)
    rng = np.random.default_rng(1204)
    m = int(ps[-1])
    bx = r_fp.x.cpu().numpy() + rng.normal(0.0, 0.02 * h, m)
    by = r_fp.y.cpu().numpy() + rng.normal(0.0, 0.02 * h, m)
    rr = np.hypot(bx, by)
    bx, by = np.where(rr > 1, bx / rr, bx), np.where(rr > 1, by / rr, by)
    sxt, syt = torch.tensor(bx, device=xt.device), torch.tensor(by, device=xt.device)
    tb_mix, rb_mix = run(ps, ids, MIXED, sxt, syt)
    tb_fp, rb_fp = run(ps, ids, FP64, sxt, syt)
    brel, bdisp = agree(ps, rb_mix, rb_fp)
    keep = np.nonzero((brel <= 1e-12) & (bdisp <= 1e-3))[0]
    eq = {"patches_same_minimum": int(keep.size), "patches_tried": subset}
    if keep.size:
        pk, ik, sel = sub_batch(ps, ids, keep)
        kx, ky = sxt[sel].contiguous(), syt[sel].contiguous()
        te_mix, re_mix = run(pk, ik, MIXED, kx, ky)
        te_fp, re_fp = run(pk, ik, FP64, kx, ky)
        erel, edisp = agree(pk, re_mix, re_fp)
        ok = (erel <= 1e-12) & (edisp <= 1e-3)
        eq.update({"mixed_s": te_mix, "fp64_s": te_fp, "speedup_at_equal_E": te_fp / te_mix,
                   "rerun_patches_within_1e-12": int(ok.sum()), "rerun_patches": int(keep.size),
                   "max_rel_energy_diff": float(erel.max()), "status_mixed": st(re_mix),
                   "status_fp64": st(re_fp)})
    return {
        "workload": f"N={n} warped lattice (sigma 0.02 h); 256 patches of the k nearest charges to "
                    f"seeded centres, k ~ U{{200..5000}} (total {int(ptr[-1])} actives); start = snapshot; "
                    f"gtol 1e-3 on the exact FP64 reduced gradient",
        "mixed_s_per_cycle_256": t_all,
        "mixed_status_256": st(r_all),
        "mixed_exact_passes_mean_256": float(r_all.iters[:, 1].float().mean().item()),
        "fp64_s_256": t_all_fp,
        "fp64_status_256": st(r_all_fp),
        "fp64_newton_steps_mean_256": float(r_all_fp.polish[:, 0].float().mean().item()),
        "fp64_exact_passes_mean_256": float(r_all_fp.iters[:, 1].float().mean().item()),
        "speedup_256_not_at_equal_E": t_all_fp / t_all,
        "same_minimum_patches_256": int(same256.sum()),
        "median_rel_energy_diff_256": float(np.median(rel256)),
        "subset_patches": subset,
        "subset_mixed_s": t_mix,
        "subset_fp64_s": t_fp,
        "subset_fp64_lbfgs_s": t_fp_lb,
        "subset_status": {"mixed": st(r_mix), "fp64": st(r_fp), "fp64_lbfgs": st(r_fp_lb)},
        "ablation_fp64_model_s": t_abl,
        "ablation_status": st(r_abl),
        "equal_E": dict(eq, start="the plain path's endpoints of the subset, kicked by N(0, (0.02 h)^2) "
                                  "per coordinate; speedup from the rerun of the patches that agreed",
                        all_subset_mixed_s=tb_mix, all_subset_fp64_s=tb_fp,
                        all_subset_speedup_not_at_equal_E=tb_fp / tb_mix,
                        all_subset_patches_disagreeing=int(subset - keep.size)),
    }


def relax_tuning(xt, yt, dev, n, defect_T):
    """relax_autotune on workload 4's batch and, in an untimed warm-up
    defect-targeted cycle, on the first batch of each size class (log2 of its
    total actives); returns the choices."""
    import torch
    from paper_2609_24722_amd import MIXED, workloads as W
    from paper_2609_24722_amd import relax as R
    from paper_2609_24722_amd.cycle import defect_cycle
    centres, sizes = W.patch_draws(n, 256, 200, 5000, 1104)
    ptr, idx = R.build_patches(xt, yt, centres, sizes)
    choices = {"workload4": R.relax_autotune(xt, yt, ptr, idx, precision=MIXED, gtol=1e-3)[:4]}
    x, y = W.workload(3, n)
    cx = torch.tensor(x, device=dev)
    cy = torch.tensor(y, device=dev)
    seen = {}

    def tune(b, sel, zx, zy, rz, pp, ii):
        key = int(pp[-1]).bit_length() - 1
        if key not in seen:
            seen[key] = R.relax_autotune(cx, cy, pp, ii, precision=MIXED, gtol=1e-3)[:4]

    defect_cycle(cx, cy, T=defect_T, precision=MIXED, inspect=tune)
    choices["defect_cycle_by_log2_actives"] = {str(k): v for k, v in sorted(seen.items())}
    return choices


def relax_only(dev, prec):
    """One relax_subdomains call on the 256 patches of workload 4 (for profiles)."""
    import numpy as np
    import torch
    from paper_2609_24722_amd import workloads as W
    from paper_2609_24722_amd import relax as R
    x, y = W.workload(4)
    xt = torch.tensor(x, device=dev)
    yt = torch.tensor(y, device=dev)
    centres, sizes = W.patch_draws(x.size, 256, 200, 5000, 1104)
    ptr, idx = R.build_patches(xt, yt, centres, sizes)
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = R.relax_subdomains(xt, yt, ptr, idx, precision=prec, gtol=1e-3)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    it = r.iters.cpu().numpy()
    print(json.dumps({"relax_precision": "mixed" if prec else "fp64", "patches": 256,
                      "actives": int(ptr[-1]), "seconds": dt,
                      "status": np.bincount(r.status.cpu().numpy(), minlength=4).tolist(),
                      "iterations_mean": float(it[:, 0].mean()), "iterations_max": int(it[:, 0].max()),
                      "exact_passes_mean": float(it[:, 1].mean())}), flush=True)


def copy_probe(dev):
    """A plain device-to-device copy of 512 MiB, three times (for counters)."""
    import torch
    a = torch.empty(64 << 20, dtype=torch.float64, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read_per_launch": a.numel() * 8,
                      "copy_probe_bytes_written_per_launch": a.numel() * 8}), flush=True)


def cycles_mode(dev, cycles, n, precision):
    import torch
    from paper_2609_24722_amd import workloads as W
    from paper_2609_24722_amd.cycle import perturb_relax_cycles
    x, y = W.workload(5, n)
    xt = torch.tensor(x, device=dev)
    yt = torch.tensor(y, device=dev)
    log = lambda r: print(json.dumps(r), flush=True)
    recs = perturb_relax_cycles(xt, yt, cycles, precision=precision, log=log)
    drift = max(abs(r["energy"] - r["tracked_energy"]) / r["energy"] for r in recs)
    print(json.dumps({"cycles": cycles, "n": n, "precision": "mixed" if precision else "fp64",
                      "final_energy": recs[-1]["energy"],
                      "seconds_per_cycle": recs[-1]["wall_s"] / cycles, "max_tracked_drift_rel": drift}),
          flush=True)


def defect_cycle_run(dev, n, kappa, precision, T=1000, log=None):
    """One defect-targeted cycle of T zones (Sec. II.C) on fresh positions of
    the N-charge lattice; returns its summary without the per-batch list."""
    import torch
    from paper_2609_24722_amd import workloads as W
    from paper_2609_24722_amd.cycle import defect_cycle
    from paper_2609_24722_amd import structure as ST
    x, y = W.workload(3, n)
    xt = torch.tensor(x, device=dev)
    yt = torch.tensor(y, device=dev)
    before = ST.summary(xt, yt)
    out = defect_cycle(xt, yt, T=T, kappa=kappa, precision=precision, log=log)
    after = ST.summary(xt, yt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ST.voronoi(xt, yt)
    torch.cuda.synchronize()
    vor_ms = (time.perf_counter() - t0) * 1e3
    for d in (before, after):
        d.pop("radial_counts")
    out["structure"] = {"before": before, "after": after, "voronoi_ms": vor_ms,
                        "note": "Voronoi coordination fractions over charges with bounded cells (hull excluded)"}
    recs = out.pop("batch_records")
    out["batch_zones_first_last"] = [recs[0]["zones"], recs[-1]["zones"]] if recs else []
    out["workload"] = (f"N={n} warped lattice (sigma 0.02 h, seed 1003); T={T} zones, kappa={kappa}, "
                       f"p_defect 0.8, radius triangle wave (period 250) from sqrt(200/N) to sqrt(4000/N), "
                       f"first-fit batches of mutually apart zones (gap 2h), relax gtol 1e-3, "
                       f"{'mixed' if precision else 'fp64'}")
    out["rel_energy_drop"] = (out["E_start"] - out["E_end"]) / out["E_start"]
    out["tracked_minus_fresh_rel"] = (out["tracked_energy"] - out["E_end"]) / out["E_end"]
    out["context_paper_first_cycle_hours_cpu"] = 31
    return out


def border_sweep(dev, n, T, precision, offsets=(-2, -1, 0, 1, 2)):
    """Table-I-style sweep: one defect-targeted cycle per boundary population
    N_b = Eq. 4's value + offset (border-interior split, sigma ramped from
    Eq. 5's value to 1 over the cycle), and one under the hard wall, all from
    the same start (lattice workload 5 at this N)."""
    import torch
    from paper_2609_24722_amd import border as B
    from paper_2609_24722_amd import workloads as W
    from paper_2609_24722_amd.cycle import defect_cycle
    x, y = W.workload(5, n)
    nb0 = B.boundary_count(n)
    rows = []
    for off in (None,) + tuple(offsets):
        xt = torch.tensor(x, device=dev)
        yt = torch.tensor(y, device=dev)
        nb = None if off is None else nb0 + off
        out = defect_cycle(xt, yt, T=T, precision=precision, border_nb=nb)
        out.pop("batch_records")
        row = {"n": n, "N_b": nb, "N_core": None if nb is None else n - nb, "E_start": out["E_start"],
               "E_end": out["E_end"], "wall_s": out["wall_s"], "batches": out["batches"],
               "committed": out["committed"], "sigma_start": out["sigma_start"],
               "tracked_minus_fresh_rel": (out["tracked_energy"] - out["E_end"]) / out["E_end"]}
        rows.append(row)
        print(json.dumps(row), flush=True)
    print(json.dumps({"border_sweep": rows, "N_b_eq4": nb0, "T": T,
                      "precision": "mixed" if precision else "fp64"}), flush=True)


def pair_scaling(dev, sizes, lib, hip):
    """The mixed energy+forces call on the warped lattice at each N: call and
    pair-kernel times (the kernel interval spans every batch of partial sums
    and their reductions where one call needs several), pair rate and the
    roofline fraction of 13 flops per ordered pair."""
    import torch
    from paper_2609_24722_amd import MIXED, ops
    from paper_2609_24722_amd import workloads as W
    for n in sizes:
        x, y = W.workload(3, n)
        xt = torch.tensor(x, device=dev)
        yt = torch.tensor(y, device=dev)
        steps = 5 if n > 200000 else 20
        call_ms, kern_ms = timed(lambda: ops.forces(xt, yt, MIXED), steps, 2, lib, hip)
        pairs = x.size * (x.size - 1)
        print(json.dumps({"n": x.size, "call_ms": call_ms, "kernel_ms": kern_ms,
                          "pairs_per_s": pairs / (call_ms * 1e-3),
                          "frac": FLOPS_EF * pairs / (kern_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS}),
              flush=True)
        del xt, yt
        torch.cuda.empty_cache()


def traffic_from_profiles():
    """HBM bytes per launch of the pair kernel from the committed counter
    summary, if it matches the current kernel build; else None."""
    p = os.path.join(ROOT, "profiles", "k_sym_forces_n100000_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
        src = open(os.path.join(ROOT, "paper_2609_24722_amd", "csrc", "pairs.hip"), "rb").read()
        import hashlib
        if d.get("pairs_hip_sha256") != hashlib.sha256(src).hexdigest():
            return None
        return d.get("traffic_bytes_per_launch")
    except Exception:
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # a cold GPU takes about ten calls of this size to reach its steady clock
    # (the kernel trace shows 2.08 ms falling to 1.83 ms per call)
    ap.add_argument("--warmup", type=int, default=15)
    ap.add_argument("--n", type=int, default=100000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-relax", action="store_true")
    ap.add_argument("--relax-subset", type=int, default=64)
    ap.add_argument("--cycles", type=int, default=0)
    ap.add_argument("--cycle-n", type=int, default=40000)
    ap.add_argument("--cycle-precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--tune", action="store_true",
                    help="pick the pair pass's launch shape with coulomb_autotune before timing")
    ap.add_argument("--no-defect", action="store_true", help="skip the defect-targeted cycle")
    ap.add_argument("--defect-only", choices=["mixed", "fp64"], default=None,
                    help="run one defect-targeted cycle (N=--n, T=--defect-T) and exit")
    ap.add_argument("--defect-T", type=int, default=1000)
    ap.add_argument("--defect-kappa", type=float, default=-1.0)
    ap.add_argument("--border-sweep", type=int, default=0, metavar="N",
                    help="one defect-targeted cycle per N_b around Eq. 4 (border-interior split) at N "
                         "charges, plus the hard wall, and exit")
    ap.add_argument("--tune-relax", action="store_true",
                    help="pick relax schedules with relax_autotune (workload 4, and per batch size class "
                         "in an untimed warm-up cycle) before the relax and cycle measurements")
    ap.add_argument("--pair-scaling", type=str, default=None,
                    help="comma-separated N: time the mixed energy+forces call at each N "
                         "(20 timed calls after 2 warm-ups, 5 above N = 2e5), one JSON line per N")
    ap.add_argument("--relax-only", choices=["mixed", "fp64"], default=None,
                    help="time one relax_subdomains call on the 256 patches of workload 4 and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the all-pairs pass would shard by i-range across "
              "GPUs, but no multi-GPU path is built; run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2609_24722_amd import FP64, MIXED, ops, workloads as W

    dev = torch.device("cuda:0")
    if args.copy_probe:
        copy_probe(dev)
        return
    if args.cycles > 0:
        cycles_mode(dev, args.cycles, args.cycle_n, MIXED if args.cycle_precision == "mixed" else FP64)
        return
    if args.relax_only:
        relax_only(dev, MIXED if args.relax_only == "mixed" else FP64)
        return
    if args.border_sweep:
        border_sweep(dev, args.border_sweep, args.defect_T, MIXED)
        return
    if args.defect_only:
        log = lambda r: print(json.dumps(r), flush=True)
        print(json.dumps(defect_cycle_run(dev, args.n, args.defect_kappa,
                                          MIXED if args.defect_only == "mixed" else FP64,
                                          args.defect_T, log)), flush=True)
        return
    lib = ops.lib()
    lib.coulomb_set_kernel_events.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.coulomb_set_kernel_events.restype = None
    hip = hip_runtime()
    if args.pair_scaling:
        pair_scaling(dev, [int(float(v)) for v in args.pair_scaling.split(",")], lib, hip)
        return

    x, y = W.workload(3, args.n)
    n = x.size
    pairs = n * (n - 1)
    xt = torch.tensor(x, device=dev)
    yt = torch.tensor(y, device=dev)
    vx, vy = W.unit_vector(n, 1103)
    vxt = torch.tensor(vx, device=dev)
    vyt = torch.tensor(vy, device=dev)
    torch.cuda.synchronize()
    # launch shape of the pair pass: the library default, or the tuner's pick
    shape = ops.autotune(xt, yt, ops.OP_FORCES) if args.tune else (0, 8, 8)

    step_ms, kern_ms = timed(lambda: ops.forces(xt, yt, MIXED), args.steps, args.warmup, lib, hip)
    spread = dict(timed.last)
    value = pairs / (step_ms * 1e-3)
    achieved = FLOPS_EF * pairs / (kern_ms * 1e-3) / 1e12
    out = {
        "metric": "pair-interactions/s (E+F, N=1e5) & subdomain relax s/cycle at equal E vs FP64",
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"N={n} charges, warped triangular lattice with Gaussian jitter 0.02 h "
                        f"(seed 1003); one fused energy+force evaluation, FP32 pairs on block-relative "
                        f"coordinates folded into FP64",
            "n": n,
            "pairs_per_step": pairs,
            "pair_convention": "ordered, N(N-1); each unordered pair is evaluated once",
            "precision": "mixed",
        },
        "roofline": {
            "bound": "alu",
            "launch_shape": {"waves_per_workgroup": shape[1], "offsets_per_chunk": shape[2],
                             "tuned": bool(args.tune)},
            "achieved": achieved,
            "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS,
            "traffic": traffic_from_profiles(),
            "kernel": "cd::k_sym<1,false> (energy+forces)",
            "kernel_ms": kern_ms,
            "timing_spread": spread,
            "flops_per_pair": FLOPS_EF,
            "peak_note": ("157.3 TFLOP/s assumes packed FP32 (two FMAs per lane per instruction), "
                          "which these kernels do not use; an all-FMA stream of unpacked FP32 "
                          f"instructions reaches about {FP32_UNPACKED_FMA_TFLOPS} TFLOP/s on gfx950 "
                          "(measured issue rate, one instruction per four clocks per SIMD)"),
            "frac_of_unpacked_fma": achieved / FP32_UNPACKED_FMA_TFLOPS,
            # each unordered pair is evaluated once, with about 17 flops of work
            # (2 sub, 3 r^2, rsqrt, add, 2 r^-3, 4 FMA for i, 4 FMA for j)
            "flops_executed_per_unordered_pair": FLOPS_EF_EXEC,
            "frac_executed": FLOPS_EF_EXEC * (pairs / 2) / (kern_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS,
        },
    }
    if not args.no_extra:
        extra = {}
        s, k = timed(lambda: ops.forces(xt, yt, FP64), 3, 1, lib, hip)
        extra["fp64_forces"] = {"pairs_per_s": pairs / (s * 1e-3), "ms": s, "kernel_ms": k,
                                "alg_tflops": FLOPS_EF * pairs / (k * 1e-3) / 1e12}
        for name, prec in (("mixed_hvp", MIXED), ("fp64_hvp", FP64)):
            s, k = timed(lambda: ops.hvp(xt, yt, vxt, vyt, prec), 5 if prec == MIXED else 3, 1, lib, hip)
            extra[name] = {"pairs_per_s": pairs / (s * 1e-3), "ms": s, "kernel_ms": k,
                           "alg_tflops": FLOPS_HVP * pairs / (k * 1e-3) / 1e12}
        s, k = timed(lambda: ops.energy(xt, yt, MIXED), 5, 1, lib, hip)
        extra["mixed_energy"] = {"pairs_per_s": pairs / (s * 1e-3), "ms": s, "kernel_ms": k}
        # Riesz-s (1/r^s pairs): the pair term needs log2 and exp2 instead of one rsqrt
        for name, prec, sv, reps in (("riesz_s2_mixed", MIXED, 2.0, 5), ("riesz_s3_mixed", MIXED, 3.0, 5),
                                     ("riesz_s2_fp64", FP64, 2.0, 2), ("riesz_s1.7_fp64", FP64, 1.7, 2)):
            s, k = timed(lambda: ops.riesz(xt, yt, sv, prec), reps, 1, lib, hip)
            extra[name] = {"pairs_per_s": pairs / (s * 1e-3), "ms": s, "kernel_ms": k,
                           "alg_tflops": FLOPS_RIESZ * pairs / (k * 1e-3) / 1e12}
        out["extra"] = extra
    if not args.no_relax:
        tuned = relax_tuning(xt, yt, dev, n, args.defect_T) if args.tune_relax else None
        out["relax"] = relax_comparison(xt, yt, args.relax_subset)
        out["relax"]["schedule"] = tuned if tuned else "library default (not tuned)"
    if not args.no_relax and not args.no_defect:  # --no-relax skips every relax measurement
        progress("defect-targeted cycle")
        out["defect_cycle"] = defect_cycle_run(dev, n, args.defect_kappa, MIXED, args.defect_T)
        progress(f"defect-targeted cycle: {out['defect_cycle']['wall_s']:.2f} s")
    if not args.no_cpu:
        progress("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(x, y)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
