"""Plant plausible mistakes in a copy of the oracle and check that the pins catch them.

Each mutant is a one-expression edit of oracle/ism_oracle.c compiled into a
temporary library; the pins of test_oracle_pins.py, test_oracle_lut.py and
test_oracle_polar.py are then run against it and at least one must fail. The oracle itself is never modified.
"""
import inspect
import os
import subprocess

import pytest

from oracle import oracle as oracle_module

import tests.test_oracle_lut as lut_pins
import tests.test_oracle_pins as pins
import tests.test_oracle_polar as polar_pins

MUTANTS = {
    "swap_wall_x0_x1": ("return ipow(b0, e0) * ipow(b1, e1);", "return ipow(b1, e0) * ipow(b0, e1);"),
    "eq1_parity": ("if (n % 2 == 0) return n * L + s;", "if (n % 2 != 0) return n * L + s;"),
    "delay_c_over_fs": ("im.x = im.d / room->c * room->fs;", "im.x = im.d * room->c / room->fs;"),
    "hann_half_width": ("cos(2.0 * PI * v / W)", "cos(PI * v / W)"),
    "amp_2pi": ("im.A = g / (4.0 * PI * im.d);", "im.A = g / (2.0 * PI * im.d);"),
    "sinc_cutoff_fs": ("sin(PI * v) / (PI * v)", "sin(2.0 * PI * v) / (2.0 * PI * v)"),
    "exponent_floor_ceil": ("int e0 = abs((int)floor(n / 2.0));", "int e0 = abs((int)ceil(n / 2.0));"),
    "distance_to_source": ("double diff = rcv[a] - p;", "double diff = rcv[a] - src[a];"),
    "window_drops_edges": ("if (fabs(v) < W / 2.0)\n", "if (fabs(v) < W / 2.0 - 1.0)\n"),
    "lattice_upper_floor": ("static int lat_hi(int N) { return (int)ceil(N / 2.0); }",
                            "static int lat_hi(int N) { return (int)floor(N / 2.0); }"),
    "zero_pow_zero": ("for (int i = 0; i < e; ++i) r *= b;", "for (int i = 0; i <= e; ++i) r *= b;"),
    "sabine_constant": ("double alpha = 0.161 * V / (S * t60);", "double alpha = 0.163 * V / (S * t60);"),
    "sabine_alpha_linear": ("double b = sqrt(1.0 - alpha);", "double b = 1.0 - alpha;"),
    "n_samples_floor": ("return (int64_t)ceil(v);", "return (int64_t)floor(v);"),
    "n_img_formula": ("n_out[a] = 4 * (int)ceil(c * t / (2.0 * L[a])) + 2;",
                      "n_out[a] = 2 * (int)ceil(c * t / (2.0 * L[a])) + 2;"),
    "sign_of_odd_image": ("return (n + 1) * L - s;", "return (n + 1) * L + s;"),
    # table taps (Sec. 3.5, Eq. (9))
    "lut_nearest_entry": ("int64_t n0 = (int64_t)floor(p);", "int64_t n0 = (int64_t)floor(p + 0.5);"),
    "lut_weight_flipped": ("const double a = p - (double)n0;", "const double a = 1.0 - (p - (double)n0);"),
    "lut_window_width": ("cos(2.0 * PI * (double)n / (q * W))", "cos(2.0 * PI * (double)n / W)"),
    "lut_sinc_scale": ("double u = (double)n / q;", "double u = (double)n / (q - 1);"),
    # directional receivers
    "polar_direction_sign": ("im.to_image[a] = -diff;", "im.to_image[a] = diff;"),
    "polar_coefficients_swapped": ("im.A *= pattern_a + (1.0 - pattern_a) * cos_theta;",
                                   "im.A *= (1.0 - pattern_a) + pattern_a * cos_theta;"),
    "polar_no_normalisation": ("/ (im.d * onorm);", "/ im.d;"),
}


def _pin_functions():
    out = []
    members = [m for mod in (pins, lut_pins, polar_pins) for m in inspect.getmembers(mod, inspect.isfunction)]
    for name, fn in members:
        if not name.startswith("test_"):
            continue
        params = getattr(fn, "pytestmark", [])
        cases = [{}]
        for m in params:
            if m.name == "parametrize":
                argnames = [a.strip() for a in m.args[0].split(",")]
                cases = [dict(zip(argnames, v if isinstance(v, tuple) and len(argnames) > 1 else (v,)))
                         for v in m.args[1]]
        for case in cases:
            out.append((name, fn, case))
    return out


@pytest.fixture(scope="module")
def mutant_dir(tmp_path_factory):
    return tmp_path_factory.mktemp("oracle_mutants")


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_pins_catch_mutant(mutant, mutant_dir, monkeypatch):
    src = open(os.path.join(os.path.dirname(oracle_module.__file__), "ism_oracle.c")).read()
    old, new = MUTANTS[mutant]
    assert src.count(old) == 1, f"mutation site for {mutant} not unique"
    c_path = mutant_dir / f"{mutant}.c"
    c_path.write_text(src.replace(old, new))
    so_path = mutant_dir / f"lib_{mutant}.so"
    inc = os.path.dirname(oracle_module.__file__)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-I", inc, str(c_path),
                           "-o", str(so_path), "-lm"])
    monkeypatch.setattr(oracle_module, "_LIB", str(so_path))
    monkeypatch.setattr(oracle_module, "_lib", None)
    failed = []
    for name, fn, case in _pin_functions():
        try:
            fn(oracle_module, **case)
        except (AssertionError, ValueError, ZeroDivisionError, FloatingPointError, IndexError) as e:
            failed.append(name)
    monkeypatch.setattr(oracle_module, "_lib", None)
    assert failed, f"no pin caught mutant {mutant}"
