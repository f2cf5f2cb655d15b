"""Selectivity sweep with the oracle only: PSNR of WASABI against the circ()-windowed Eq.(1) sum
as a function of gamma (Sec. 2, step 1: N_r = gamma pi R^2).  Writes the table and the smallest
gamma on a 0.01 grid whose PSNR reaches 40 dB.

  2048:  the 2048^2, N = 10^4, 64-plane, L = 3 workload -> tests/golden/gamma40_2048.txt.  PSNR
         over the 512 x 512 window at pixel (768, 768).
  65536: the 65536^2, N = 10^6 height-field, 256-plane, L = 4 workload ->
         tests/golden/gamma40_65536.txt.  PSNR pooled over four seeded 2^L-aligned 512 x 512
         windows (peak power of the reference over all of them, mean error power over all of them);
         a window is given the points whose PSF table can reach it, the others add nothing to it.

PSNR = 10 log10(max|u_ref|^2 / mean|u - u_ref|^2) (Haar windows are exact, so a window equals that
part of the full hologram); u_ref is the FP64 direct sum with the same plane-snapped depths and
grid positions.

Run:  python oracle/gamma_sweep.py [2048|65536]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import WASABI_2048, WASABI_65536, grid_points, height_field_points  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "gamma40_2048.txt")
OUT_65536 = os.path.join(ROOT, "tests", "golden", "gamma40_65536.txt")
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


def near(q, x0, y0, w, reach):
    keep = (q.x >= x0 - reach) & (q.x < x0 + w + reach) & (q.y >= y0 - reach) & (q.y < y0 + w + reach)
    return oracle.Quantized(q.x[keep], q.y[keep], q.d[keep], q.a[keep])


def windows_65536(side, B, k=4, seed=21):
    rng = np.random.default_rng(seed)
    return [(int(v[0]) * B, int(v[1]) * B) for v in rng.integers(0, (side - SIDE) // B, (k, 2))]


def main_65536():
    w = WASABI_65536
    B = 1 << w["levels"]
    pts = height_field_points(w["seed"], w["n"], w["nx"], B, w["z_lo"], w["z_hi"])
    wins = windows_65536(w["nx"], B)
    reach = w["max_window"] // 2 + B
    prm1 = oracle.LutParams(n_depth=w["n_depth"], levels=w["levels"], gamma=1.0, max_window=w["max_window"])
    # the direct reference needs only the plane depths, not the tables: geometry of the planes
    z = oracle.lut_geometry(prm1)[0]
    q = oracle.quantize(pts, prm1)
    t0 = time.time()
    refs = []
    for x0, y0 in wins:
        qn = near(q, x0, y0, SIDE, reach)
        ok = qn.d >= 0
        sn = np.stack([qn.x[ok] * prm1.pitch, qn.y[ok] * prm1.pitch, z[qn.d[ok]], qn.a[ok]], axis=1)
        refs.append(oracle.direct(np.ascontiguousarray(sn), SIDE, SIDE, x0, y0, window=oracle.CIRC))
    print("references %.1fs" % (time.time() - t0), flush=True)
    peak = max(float(np.max(np.abs(r)) ** 2) for r in refs)

    def psnr_at(gamma):
        prm = oracle.LutParams(n_depth=w["n_depth"], levels=w["levels"], gamma=gamma, max_window=w["max_window"])
        lut = oracle.build_lut(prm)
        num = 0.0
        for (x0, y0), ref in zip(wins, refs):
            u = oracle.wasabi(lut, near(q, x0, y0, SIDE, reach), x0, y0, SIDE, SIDE)
            num += float(np.sum(np.abs(u - ref) ** 2))
        mse = num / (len(refs) * SIDE * SIDE)
        return 10.0 * np.log10(peak / mse), int(lut.off[-1])

    rows = []
    for g in [0.6, 0.7, 0.75, 0.8, 0.85, 0.9]:
        p, tot = psnr_at(g)
        rows.append((g, p, tot))
        print("gamma %.2f  psnr %.2f dB  entries %d" % (g, p, tot), flush=True)
    lo = max(g for g, p, _ in rows if p < 40.0)
    hi = min(g for g, p, _ in rows if p >= 40.0)
    g = round(lo + 0.01, 2)
    while g < hi - 1e-9:
        p, tot = psnr_at(g)
        rows.append((g, p, tot))
        print("gamma %.2f  psnr %.2f dB  entries %d" % (g, p, tot), flush=True)
        if p >= 40.0:
            break
        g = round(g + 0.01, 2)
    rows.sort()
    g40 = min(g for g, p, _ in rows if p >= 40.0)
    with open(OUT_65536, "w") as f:
        f.write("# Selectivity vs PSNR, written by oracle/gamma_sweep.py 65536 (oracle only).\n")
        f.write("# Workload: 65536^2, N = 10^6 height-field points (seed 0), z in [0.1, 1.5] mm,\n")
        f.write("# 256 planes, Haar L = 4, FP32 LUT values; PSNR pooled over the 512^2 windows at\n")
        f.write("# %s against the FP64 circ()-windowed Eq.(1) sum with the same snapped inputs.\n"
                % " ".join("(%d, %d)" % xy for xy in wins))
        f.write("# smallest gamma (0.01 grid) with PSNR >= 40 dB:\n")
        f.write("%.2f\n" % g40)
        f.write("# columns: gamma psnr_db lut_entries\n")
        for g, p, tot in rows:
            f.write("%.2f %.3f %d\n" % (g, p, tot))
    print("gamma40 =", g40)


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "65536":
        main_65536()
    else:
        main()
