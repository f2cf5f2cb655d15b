"""Selectivity sweep with the oracle only: PSNR of WASABI against the circ()-windowed Eq.(1) sum
as a function of gamma (Sec. 2, step 1: N_r = gamma pi R^2), on the 2048^2, N = 10^4, 64-plane,
L = 3 workload.  Writes tests/golden/gamma40_2048.txt with the table and the smallest gamma on a
0.01 grid whose PSNR reaches 40 dB.

PSNR = 10 log10(max|u_ref|^2 / mean|u - u_ref|^2) over a 512 x 512 window at pixel (768, 768)
(Haar windows are exact, so the window equals that part of the full hologram); u_ref is the FP64
direct sum with the same plane-snapped depths and grid positions.

Run:  python oracle/gamma_sweep.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import WASABI_2048, grid_points  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "gamma40_2048.txt")
X0, Y0, SIDE = 768, 768, 512


def psnr_at(gamma, pts, ref):
    w = WASABI_2048
    prm = oracle.LutParams(n_depth=w["n_depth"], levels=w["levels"], gamma=gamma,
                           max_window=w["max_window"])
    lut = oracle.build_lut(prm)
    q = oracle.quantize(pts, prm)
    u = oracle.wasabi(lut, q, X0, Y0, SIDE, SIDE)
    return oracle.psnr(u, ref), int(lut.off[-1])


def main():
    w = WASABI_2048
    pts = grid_points(w["seed"], w["n"], w["nx"], w["ny"], 8, w["z_lo"], w["z_hi"])
    prm = oracle.LutParams(n_depth=w["n_depth"], levels=w["levels"], gamma=1.0,
                           max_window=w["max_window"])
    lut1 = oracle.build_lut(prm)
    snapped = oracle.snapped_points(oracle.quantize(pts, prm), lut1)
    t0 = time.time()
    ref = oracle.direct(snapped, SIDE, SIDE, X0, Y0, window=oracle.CIRC)
    print("reference %.1fs" % (time.time() - t0), flush=True)
    rows = []
    for g in [0.05, 0.2, 0.4, 0.6, 0.8, 0.85, 0.9, 0.95]:
        p, tot = psnr_at(g, pts, ref)
        rows.append((g, p, tot))
        print("gamma %.2f  psnr %.2f dB  entries %d" % (g, p, tot), flush=True)
    lo = max(g for g, p, _ in rows if p < 40.0)
    hi = min(g for g, p, _ in rows if p >= 40.0)
    g = round(lo + 0.01, 2)
    while g < hi - 1e-9:
        p, tot = psnr_at(g, pts, ref)
        rows.append((g, p, tot))
        print("gamma %.2f  psnr %.2f dB  entries %d" % (g, p, tot), flush=True)
        if p >= 40.0:
            break
        g = round(g + 0.01, 2)
    rows.sort()
    g40 = min(g for g, p, _ in rows if p >= 40.0)
    with open(OUT, "w") as f:
        f.write("# Selectivity vs PSNR, written by oracle/gamma_sweep.py (oracle only).\n")
        f.write("# Workload: 2048^2, N = 10^4 grid points (seed 0), z in [0.1, 1.5] mm, 64 planes,\n")
        f.write("# Haar L = 3, FP32 LUT values; PSNR over the 512^2 window at (768, 768) against the\n")
        f.write("# FP64 circ()-windowed Eq.(1) sum with the same snapped inputs.\n")
        f.write("# smallest gamma (0.01 grid) with PSNR >= 40 dB:\n")
        f.write("%.2f\n" % g40)
        f.write("# columns: gamma psnr_db lut_entries\n")
        for g, p, tot in rows:
            f.write("%.2f %.3f %d\n" % (g, p, tot))
    print("gamma40 =", g40)


if __name__ == "__main__":
    main()
