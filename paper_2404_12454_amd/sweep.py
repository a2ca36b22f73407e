"""Parameter searches of Sec. 6 on the batched GBD sweep.

* ``search``: the RMS (and peak) difference between the peak-normalised GBD
  irradiance and the Airy pattern over a grid of (OF, waist/spacing ratio,
  beamlets across), all instances in one persistent launch per chunk.
* ``zone_study``: the same restricted to annular zones 0-5, 5-10 and
  10-15 lambda/D (in the focal plane lambda F), on a grid spanning
  +-15.14 lambda F with 512 x 512 pixels (the 512-pixel, 2.8 mas grid of the
  paper's search, Appendix D), reporting each zone's best overlap factor per
  beamlet count.

All numerics run in the HIP library (``gbd_eval_batch``, ``gbd_airy``).
"""
from __future__ import annotations

import json
import time

import numpy as np

from . import Context, beamlets_from_scene, gbd_airy, gbd_eval_batch, plane_from_scene, scenes


def search(ctx: Context, grid, npix=256, span=8.0, zones_lamF=None, chunk=600):
    """grid: rows (OF, q, n_across).  Returns [n, 2 + n_zones] metrics and seconds."""
    grid = np.asarray(grid, np.float64)
    nz = 0 if zones_lamF is None else len(zones_lamF) - 1
    out = np.zeros((len(grid), 2 + nz))
    airy = None
    t = 0.0
    for s in range(0, len(grid), chunk):
        rows = grid[s:s + chunk]
        sc = [scenes.airy_scene(int(na), OF=float(of), q=float(q), npix=npix, half_span_lamF=span)
              for of, q, na in rows]
        bs = [beamlets_from_scene(ctx, x) for x in sc]
        ps = [plane_from_scene(ctx, x) for x in sc]
        edges = None
        if zones_lamF is not None:
            lamF = sc[0].lam * sc[0].meta["fnum"]
            edges = np.asarray(zones_lamF, np.float64) * lamF
        if airy is None:
            m = sc[0].meta
            airy = gbd_airy(ctx, ps[0], m["D"], m["f"], sc[0].lam)
        t0 = time.perf_counter()
        metrics, _ = gbd_eval_batch(ctx, bs, ps, airy=airy, zone_edges=edges)
        t += time.perf_counter() - t0
        out[s:s + len(rows)] = metrics
    return out, t


def zone_study(ctx: Context = None, of_values=None, nacross=scenes.SWEEP_NACROSS, npix=512, span=15.14):
    ctx = ctx or Context(0)
    of_values = np.round(np.linspace(1.0, 2.0, 21), 3) if of_values is None else of_values
    grid = [(of, 1.0, na) for na in nacross for of in of_values]
    zones = [0.0, 5.0, 10.0, 15.0]
    m, secs = search(ctx, grid, npix=npix, span=span, zones_lamF=zones)
    rec = {"instances": len(grid), "seconds": secs, "npix": npix, "span_lamF": span, "zones_lamF": zones,
           "pairs": int(sum(scenes.pupil_grid(int(na), 10e-3)[0].shape[0] for _, _, na in grid) * npix * npix)}
    table = {}
    for k, name in enumerate(["all", "0-5", "5-10", "10-15"]):
        col = 0 if k == 0 else 1 + k
        best = {}
        for na in nacross:
            idx = [i for i, g in enumerate(grid) if g[2] == na]
            j = idx[int(np.argmin(m[idx, col]))]
            best[int(na)] = {"OF": float(grid[j][0]), "rms": float(m[j, col])}
        j = int(np.argmin(m[:, col]))
        table[name] = {"best_overall": {"OF": float(grid[j][0]), "n_across": int(grid[j][2]),
                                        "rms": float(m[j, col])}, "best_OF_per_n_across": best}
    rec["zones"] = table
    return rec


if __name__ == "__main__":
    print(json.dumps(zone_study()), flush=True)
