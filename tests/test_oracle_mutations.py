"""The oracle's pins catch plausible mistakes in the oracle.

Each case plants one mistake in a copy of oracle/oracle.c (a dropped term, a wrong sign, a
transposed operand, an off-by-one boundary), compiles it, and runs the oracle pin suite
(tests/test_oracle_*.py) against that library in a subprocess.  The suite must fail for every
mutant, and pass for the unmodified copy compiled the same way (the control, which shows that the
override reaches the oracle).  Nothing here changes the committed oracle.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")
PINS = sorted(os.path.join(ROOT, "tests", f) for f in os.listdir(os.path.join(ROOT, "tests"))
              if f.startswith("test_oracle_") and f.endswith(".py") and f != "test_oracle_mutations.py")

# (name, text in oracle.c, replacement); each text must occur exactly once.
MUTATIONS = [
    # Eq.(1): phase 2 pi r / lambda with the factor 2 dropped
    ("direct_phase_half", "const double phase = 2.0 * M_PI * r / wavelength;",
     "const double phase = M_PI * r / wavelength;"),
    # Eq.(1): r = sqrt(rho^2 + z) instead of sqrt(rho^2 + z^2)
    ("direct_r_no_square", "const double r = sqrt(rho2 + z * z);", "const double r = sqrt(rho2 + z);"),
    # circ(): <= instead of the strict < of circ(c) = 1 iff c < 1
    ("direct_circ_closed", "if (!(rho2 < R * R)) continue;", "if (!(rho2 <= R * R)) continue;"),
    # planes at the cell's lower edge instead of its centre
    ("plane_at_edge", "z[d] = z_min + ((double)d + 0.5) * dz;", "z[d] = z_min + (double)d * dz;"),
    # N_r = gamma pi R (R not squared)
    ("nr_linear_in_r", "double want = ceil(gamma * M_PI * R[d] * R[d]);",
     "double want = ceil(gamma * M_PI * R[d]);"),
    # table side without the +2 margin (the disk may touch the table edge)
    ("table_margin", "int32_t need = 2 * (int32_t)floor(R[d]) + (phases ? q : 2);",
     "int32_t need = 2 * (int32_t)floor(R[d]) + (phases ? q : 0);"),
    # PSF disk of radius R/2 (W read as a radius rather than a diameter)
    ("psf_radius_half", "if (dq * dq + dr * dr < R * R) {", "if (dq * dq + dr * dr < R * R / 4.0) {"),
    # PSF table: pixels on the rim counted inside
    ("psf_circ_closed", "if (dq * dq + dr * dr < R * R) {", "if (dq * dq + dr * dr <= R * R) {"),
    # phase-table shift applied transposed
    ("psf_shift_transposed", "const int32_t cx = W / 2 + sx, cy = W / 2 + sy;",
     "const int32_t cx = W / 2 + sy, cy = W / 2 + sx;"),
    # forward Haar: H band gets V's sign pattern
    ("haar_h_is_v", "t[2 * ((int64_t)m * w + w2 + n) + ri] = (a - b + c - d) / 2.0;",
     "t[2 * ((int64_t)m * w + w2 + n) + ri] = (a + b - c - d) / 2.0;"),
    # forward Haar: 1/4 per level (not orthonormal)
    ("haar_scale", "t[2 * ((int64_t)m * w + n) + ri] = (a + b + c + d) / 2.0;",
     "t[2 * ((int64_t)m * w + n) + ri] = (a + b + c + d) / 4.0;"),
    # inverse Haar: wrong sign on D for the pixel b
    ("ihaar_sign", "t[2 * ((int64_t)(2 * m) * w + 2 * n + 1) + ri] = (S - H + V - D) / 2.0;",
     "t[2 * ((int64_t)(2 * m) * w + 2 * n + 1) + ri] = (S - H + V + D) / 2.0;"),
    # selection strength from the real part only
    ("select_real_only", "e[k].mag2 = (float)(C[2 * k] * C[2 * k] + C[2 * k + 1] * C[2 * k + 1]);",
     "e[k].mag2 = (float)(C[2 * k] * C[2 * k]);"),
    # selection ties to the higher flat index
    ("select_ties_high", "return (a->idx > b->idx) - (a->idx < b->idx);",
     "return (a->idx < b->idx) - (a->idx > b->idx);"),
    # FP16 rounding with 10 significant bits
    ("fp16_bits", "return round_to_bits(v, 11, -13, 65504.0);", "return round_to_bits(v, 10, -13, 65504.0);"),
    # quantise: truncate to the grid instead of rounding to the nearest multiple
    ("quantize_truncates", "const double sx = B * floor(x / pitch / B + 0.5);",
     "const double sx = B * floor(x / pitch / B);"),
    # quantise: z = z_max not clamped to the last plane
    ("quantize_zmax", "if (d > n_depth - 1) d = n_depth - 1;", ""),
    # floor of a negative shift rounds towards zero
    ("floor_toward_zero", "if (r * q > v) r -= 1;", ""),
    # Eq.(2): row shift taken from the x offset (transposed operand)
    ("superpose_transposed", "const int64_t tm = m + floor_shift(oy, lev);",
     "const int64_t tm = m + floor_shift(ox, lev);"),
    # Eq.(2): H and V band codes swapped
    ("superpose_band_swap", "band = 2 * (row >= s) + (col >= s); /* 1 = H, 2 = V, 3 = D */",
     "band = (row >= s) + 2 * (col >= s);"),
    # Eq.(2): imaginary part subtracted
    ("superpose_im_sign", "psi[2 * at + 1] += pa[j] * val[2 * k + 1];", "psi[2 * at + 1] -= pa[j] * val[2 * k + 1];"),
    # Eq.(2): amplitude dropped from the imaginary part
    ("superpose_no_amp", "psi[2 * at + 1] += pa[j] * val[2 * k + 1];", "psi[2 * at + 1] += val[2 * k + 1];"),
    # coiflet: wavelet filter without the time reversal
    ("coif_hi_no_reverse", "hi[n] = ((n & 1) ? -1.0 : 1.0) * lo[taps - 1 - n];", "hi[n] = ((n & 1) ? -1.0 : 1.0) * lo[n];"),
]


def _compile(src_text, out_dir, name):
    c = os.path.join(out_dir, name + ".c")
    so = os.path.join(out_dir, "lib" + name + ".so")
    with open(c, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", c, "-o", so, "-lm"])
    return so


def _run_pins(lib):
    env = dict(os.environ, ORACLE_LIB_OVERRIDE=lib, OMP_NUM_THREADS="1")
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *PINS],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


@pytest.fixture(scope="module")
def outcomes(tmp_path_factory):
    """Pin-suite runs of the control copy and of every mutant, several at a time."""
    out_dir = str(tmp_path_factory.mktemp("oracle_mutants"))
    text = open(SRC).read()
    cases = [("control", text)]
    for name, old, new in MUTATIONS:
        assert text.count(old) == 1, "mutation site of %s not unique in oracle.c" % name
        cases.append((name, text.replace(old, new)))

    def one(case):
        name, src = case
        return name, _run_pins(_compile(src, out_dir, name))

    workers = max(1, min(8, len(os.sched_getaffinity(0))))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return dict(ex.map(one, cases))


def test_control_copy_passes_the_pins(outcomes):
    r = outcomes["control"]
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]


@pytest.mark.parametrize("name", [m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(outcomes, name):
    r = outcomes[name]
    # a pin must fail (not an error in collection or a crash of the runner)
    assert r.returncode == 1, r.stdout[-2000:] + r.stderr[-2000:]
    assert " failed" in r.stdout
