"""Plant plausible mistakes in a copy of the oracle (CPU only) and check that
the pins catch every one of them: each mutant must make the pin suite fail."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "qtam_oracle.cpp")

# (name, original text, planted mistake)
MUTANTS = [
    ("short_idft_sign", "dft(m, Z.data(), y.data(), +1);", "dft(m, Z.data(), y.data(), -1);"),
    ("dropped_sqrt_norm",
     "const double norm = std::sqrt(static_cast<double>(m) / static_cast<double>(pl.n)) / static_cast<double>(m);",
     "const double norm = 1.0 / static_cast<double>(m);"),
    ("centre_truncated", "std::floor(r.f * T + 0.5)", "std::floor(r.f * T)"),
    ("window_scale_off_by_one",
     "const double x = static_cast<double>(c - r.s) / static_cast<double>(h);",
     "const double x = static_cast<double>(c - r.s) / static_cast<double>(h + 1);"),
    ("missing_frame_division",
     "Xh[static_cast<size_t>(b)] = acc[static_cast<size_t>(b)] / pl.P[static_cast<size_t>(b)];",
     "Xh[static_cast<size_t>(b)] = acc[static_cast<size_t>(b)];"),
    ("roll_reversed",
     "Z[static_cast<size_t>(wrap(c - r.s, m))] +=", "Z[static_cast<size_t>(wrap(r.s - c, m))] +="),
    ("inverse_scale_inverted",
     "const double scale = std::sqrt(static_cast<double>(pl.n) / static_cast<double>(m));",
     "const double scale = std::sqrt(static_cast<double>(m) / static_cast<double>(pl.n));"),
    ("hermitian_conj_missing", "F[static_cast<size_t>(n - b)] = std::conj(Xh[static_cast<size_t>(b)]);",
     "F[static_cast<size_t>(n - b)] = Xh[static_cast<size_t>(b)];"),
    ("width_not_halved", "int64_t h = static_cast<int64_t>(std::ceil(r.f * T / q)) / 2;",
     "int64_t h = static_cast<int64_t>(std::ceil(r.f * T / q));"),
    ("cap_too_narrow", "pl.l_max = 2 * g + 1;", "pl.l_max = 2 * g - 1;"),
    ("frame_not_squared", "pl.P[static_cast<size_t>(c)] += v * v;", "pl.P[static_cast<size_t>(c)] += v;"),
    ("norm_literal_by_default", "scale = 1.0 / std::sqrt(energy);", "scale = 1.0 / energy;"),
    ("radix2_twiddle_sign",
     "const double ang = sign * 2.0 * kPi * static_cast<double>(j) / static_cast<double>(len);",
     "const double ang = -sign * 2.0 * kPi * static_cast<double>(j) / static_cast<double>(len);"),
    ("synthesis_missing_1_over_n",
     "x[t] = a[static_cast<size_t>(t)].real() / static_cast<double>(n);",
     "x[t] = a[static_cast<size_t>(t)].real();"),
    ("grid_exponent_off", "static_cast<double>(k) / static_cast<double>(nrows - 1)",
     "static_cast<double>(k) / static_cast<double>(nrows)"),
    # the stop-band value replacing only exact zeros (a taper's tails below eps kept)
    ("eps_only_on_zeros", "if (eps > 0.0 && v < eps) v = eps;", "if (eps > 0.0 && v == 0.0) v = eps;"),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,orig,bad", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(name, orig, bad, tmp_path):
    src = open(SRC).read()
    assert src.count(orig) == 1, "mutation site not found exactly once: " + name
    mut = tmp_path / "mutant.cpp"
    mut.write_text(src.replace(orig, bad))
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", str(mut), "-o", str(so)])
    env = dict(os.environ, QTAM_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, "pins did not catch mutant " + name + "\n" + r.stdout[-2000:]
