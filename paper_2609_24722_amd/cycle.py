"""Cycle drivers: perturb-and-relax cycles over random subdomains, and the
paper's defect-targeted cycle (Sec. II.C).

Perturb-and-relax (``perturb_relax_cycles``), the driver loop of the
benchmark's energy-versus-time run:

Each cycle: draw patch centres and sizes (seeded), build the patches
(k nearest charges), kick their actives with Gaussian displacements, relax
all candidates in one batched call against the current configuration, and
commit the improving ones greedily with exact energy changes re-evaluated
against the configuration as it changes.  The tracked energy (start energy
plus committed changes) is compared with a from-scratch FP64 evaluation every
cycle.

Defect-targeted (``defect_cycle``): local energies and the defect list once
per cycle (steps 1-2), T zone centres and radii (step 3 and the oscillating
radius), then the zones in batches of mutually distant zones, each batch
relaxed side by side and committed greedily (step 4).

All arithmetic runs in the library; this module only sequences calls and
draws the random inputs.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import FP64, MIXED, border as B, ops, relax as R, workloads as W, zones as Z


def perturb_relax_cycles(x, y, cycles: int, n_patches: int = 64, size_lo: int = 200,
                         size_hi: int = 5000, kick: float = 0.3, seed: int = 1005,
                         precision: int = MIXED, gtol: float = 1e-3, log=None):
    """x, y: device float64 tensors, updated in place.  Returns a list of
    per-cycle records (cycle, wall_s, energy, tracked_energy, accepted, sum_dE)."""
    n = x.numel()
    h = W.spacing(n)
    torch.cuda.synchronize()
    E = ops.energy(x, y, FP64).item()
    tracked = E
    out = []
    t0 = time.perf_counter()
    for c in range(cycles):
        centres, sizes = W.patch_draws(n, n_patches, size_lo, size_hi, seed + 7919 * c)
        ptr, idx = R.build_patches(x, y, centres, sizes)
        kx, ky = W.kicks(int(ptr[-1]), kick * h, seed + 104729 + 7919 * c)
        idx_h = idx.cpu().numpy()
        sx, sy = W.kicked_starts(x.cpu().numpy(), y.cpu().numpy(), idx_h, kx, ky)
        dev = x.device
        res = R.relax_subdomains(x, y, ptr, idx, torch.tensor(sx, device=dev), torch.tensor(sy, device=dev),
                                 precision=precision, gtol=gtol)
        com, dc = R.commit_patches(x, y, ptr, idx, res.x, res.y, res.dE.cpu().numpy())
        tracked += float(dc[com == 1].sum())
        E = ops.energy(x, y, FP64).item()
        rec = {"cycle": c + 1, "wall_s": time.perf_counter() - t0, "energy": E, "tracked_energy": tracked,
               "accepted": int(com.sum()), "sum_dE": float(dc[com == 1].sum()),
               "relax_status": np.bincount(res.status.cpu().numpy(), minlength=4).tolist()}
        out.append(rec)
        if log is not None:
            log(rec)
    return out


def defect_cycle(x, y, T: int = 1000, cap: int = 256, kappa: float = -1.0, p_defect: float = 0.8,
                 n_lo: int = 200, n_hi: int = 4000, period: int = 250, gap_h: float = 2.0,
                 seed: int = 1006, precision: int = MIXED, gtol: float = 1e-3, log=None, inspect=None,
                 border_nb: int | None = None, sigma_start: float | None = None, sigma_end: float = 1.0,
                 lbfgs_m: int = 16, border_start: str = "spread", relax_kw: dict | None = None):
    """One defect-targeted cycle of T subdomain optimisations (Sec. II.C).
    x, y: device float64 tensors, updated in place.

    * Steps 1-2 once, at the start: FP64 local energies, then the defect list
      e_i > mu + kappa * sigma_e.
    * Step 3 for all T zones: centre at a defect charge with probability
      p_defect, else a uniform point of the disk.  The radius follows a
      triangle wave of `period` zones between sqrt(n_lo / N) and
      sqrt(n_hi / N), the radii that hold n_lo and n_hi charges at the mean
      density.
    * Zones are layered into batches of at most `cap` (zone_batches): zones
      of one batch are more than gap_h * h apart, and a zone that comes
      within that distance of an earlier one runs in a later batch.
    * Step 4 per batch: the zones' charges at the current positions, relaxed
      side by side against that snapshot, committed greedily with exact
      energy changes.

    * With border_nb, the border-interior split of Sec. II.B: the border_nb
      charges farthest from the centre are pinned to the unit circle, the
      others confined within sigma, which rises linearly over the cycle's
      batches from sigma_start (default Eq. 5's value) to sigma_end; at the
      start the boundary charges are spread evenly along the circle in
      their angular order (border_start "spread"; "ray": projected along
      their rays) and the others projected within sigma.
    * relax_kw: further options of relax_subdomains.

    Returns a summary dict (energies, counts, wall time, per-batch records).
    inspect(b, sel, cx, cy, rz, ptr, idx), if given, sees each batch's zones
    (host arrays of the zone indices and all T centres and radii, the packed
    active sets) before the relaxation, while x, y hold that batch's snapshot."""
    n = x.numel()
    dev = x.device
    h = W.spacing(n)
    r_lo = Z.radius_holding(n, n_lo)
    r_hi = Z.radius_holding(n, n_hi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    flags = None
    s0 = 1.0
    if border_nb is not None:
        s0 = B.sigma0(n) if sigma_start is None else float(sigma_start)
        flags = B.border_split(x, y, int(border_nb))
        if border_start == "spread":
            B.border_spread(x, y, flags)
        elif border_start != "ray":
            raise ValueError("border_start: 'spread' or 'ray'")
        B.border_project(x, y, flags, s0)
    E0, e = ops.energy(x, y, FP64, local=True)
    draws = torch.tensor(W.zone_draws(T, seed), device=dev)
    z = Z.defect_zones(x, y, e, draws, kappa, p_defect, r_lo, r_hi, 0, period)
    cx = z["cx"].cpu().numpy()
    cy = z["cy"].cpu().numpy()
    rz = z["rz"].cpu().numpy()
    ci = z["centre_idx"].cpu().numpy()
    stats = z["stats"].cpu().numpy()
    E0 = float(E0.item())
    batch, nb = Z.zone_batches(cx, cy, rz, gap_h * h, cap)
    tracked = E0
    recs = []
    committed = 0
    relaxed = 0
    actives = 0
    status = np.zeros(4, dtype=np.int64)
    for b in range(nb):
        sel = np.nonzero(batch == b)[0]
        f = dict(dtype=torch.float64, device=dev)
        ptr, idx = Z.zone_patches(x, y, torch.tensor(cx[sel], **f), torch.tensor(cy[sel], **f),
                                  torch.tensor(rz[sel], **f),
                                  capacity=int(np.sum(np.minimum(n, 2.0 * n * rz[sel] ** 2 + 64))))
        sizes = np.diff(ptr)
        keep = sizes > 0
        if not keep.any():
            continue
        if not keep.all():
            ptr = R.offsets(sizes[keep])
        if inspect is not None:
            inspect(b, sel[keep], cx, cy, rz, ptr, idx)
        sig = 0.0
        if flags is not None:
            sig = B.sigma_ramp(b, max(1, nb - 1), n, s0, sigma_end)
        res = R.relax_subdomains(x, y, ptr, idx, precision=precision, gtol=gtol, sigma=sig, boundary=flags,
                                 lbfgs_m=lbfgs_m, **(relax_kw or {}))
        com, dc = R.commit_patches(x, y, ptr, idx, res.x, res.y, res.dE.cpu().numpy())
        tracked += float(dc[com == 1].sum())
        st = np.bincount(res.status.cpu().numpy(), minlength=4)[:4]
        status += st
        committed += int(com.sum())
        relaxed += int(keep.sum())
        actives += int(ptr[-1])
        rec = {"batch": b, "zones": int(keep.sum()), "actives": int(ptr[-1]), "committed": int(com.sum()),
               "sum_dE": float(dc[com == 1].sum()), "wall_s": time.perf_counter() - t0,
               "status": st.tolist(), "sigma": sig}
        recs.append(rec)
        if log is not None:
            log(rec)
    E1 = float(ops.energy(x, y, FP64).item())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return {"T": T, "border_nb": border_nb, "sigma_start": s0 if flags is not None else None,
            "sigma_end": sigma_end if flags is not None else None, "batches": nb, "zones_relaxed": relaxed, "committed": committed,
            "actives_total": actives, "defects": int(stats[3]), "mu": float(stats[0]),
            "sigma_e": float(stats[1]), "threshold": float(stats[2]),
            "defect_centres": int((ci >= 0).sum()), "E_start": E0, "E_end": E1, "tracked_energy": tracked,
            "relax_status": status.tolist(), "wall_s": wall, "batch_records": recs}
