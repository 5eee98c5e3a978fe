"""The pins must catch plausible mistakes in the oracle.

Each case compiles a copy of ``oracle/ocd_oracle.c`` with one deliberate
mistake (a dropped term, a flipped sign, a wrong operand, a wrong label
convention...), points the oracle's loader at it, and runs the CPU pins of
``test_oracle_pins``: at least one of them must fail.  Everything here runs on
the CPU.
"""

import os
import subprocess

import pytest

import oracle
import test_oracle_fixed_pins as fpins
import test_oracle_mmse_pins as mpins
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "ocd_oracle.c")

# (name, exact text in the source, replacement)
MUTANTS = [
    ("drop p_u z_u in Alg. 1", "ip + p[k * U + u] * z[u]);", "ip);"),
    ("h instead of conj(h) in the inner product", "ip += conj(h[b]) * r[b];", "ip += h[b] * r[b];"),
    ("residual update with the wrong sign", "r[b] -= h[b] * delta;", "r[b] += h[b] * delta;"),
    ("imaginary part clipped on one side only", "if (im < -P->beta) im = -P->beta;", ""),
    ("dinv ignores the regulariser", "double di = (den > 0.0) ? 1.0 / den : 0.0;",
     "double di = (g[u] > 0.0) ? 1.0 / g[u] : 0.0;"),
    ("column norm drops the imaginary part", "acc += creal(h) * creal(h) + cimag(h) * cimag(h);",
     "acc += creal(h) * creal(h);"),
    ("LLR sign flipped", "L[b] = rho * (d0 - d1);", "L[b] = rho * (d1 - d0);"),
    ("channel gain taken as 1", "*mu = g / (g + lamK);", "*mu = 1.0;"),
    ("SINR taken as mu", "*rho = g / lamK;", "*rho = g / (g + lamK);"),
    ("BOX SINR ignores Es", "*rho = g * P->Es / P->N0;", "*rho = g / P->N0;"),
    ("default regulariser ignores Es", "(mode == MODE_BOX) ? 0.0 : N0 / Es;", "(mode == MODE_BOX) ? 0.0 : N0;"),
    ("LLR point ignores Es", "/ (mu * sqrt(Es));", "/ (mu);"),
    ("natural instead of Gray labels", "unsigned gi = (unsigned)(mi ^ (mi >> 1));", "unsigned gi = (unsigned)mi;"),
    ("Q bits before I bits", "labels[i] = (gi << half) | gq;", "labels[i] = (gq << half) | gi;"),
    ("box edge off by one level", "return (double)(M - 1) / sqrt(", "return (double)M / sqrt("),
    ("gradient drops the p_u-path of lambda", "- g[u] * di * di * creal(conj(zold[ku]) * cbar);", ";"),
    ("gradient passes clipped components", "else cre = creal(ztot);", "cre = creal(ztot);"),
    ("gradient drops -Delta_bar in z_bar", "zbar[u] = -dbar + p[ku] * cbar;", "zbar[u] = p[ku] * cbar;"),
    ("gradient Delta_bar sign", "cplx dbar = -hr;", "cplx dbar = hr;"),
    ("gradient drops the mu-path of lambda_K",
     "dlambda[K - 1] += dmu * (-g[u] / ((g[u] + lamK) * (g[u] + lamK)));", ""),
    # explicit MMSE (Sections II-B, II-E)
    ("MMSE regulariser ignores Es", "const double lam = N0 / Es;", "const double lam = N0;"),
    ("Gram matrix without the conjugate", "s += conj(Hw[i * B + b]) * Hw[j * B + b];",
     "s += Hw[i * B + b] * Hw[j * B + b];"),
    ("matched filter without the conjugate", "acc += conj(Hw[i * B + b]) * yv[b];",
     "acc += Hw[i * B + b] * yv[b];"),
    ("Cholesky pivot drops the imaginary parts", "d -= creal(l) * creal(l) + cimag(l) * cimag(l);",
     "d -= creal(l) * creal(l);"),
    ("back substitution without conj(L)", "s -= conj(Lf[k * n + i]) * Ainv[k * n + j];",
     "s -= Lf[k * n + i] * Ainv[k * n + j];"),
    ("gain from column i of A^-1", "s += Ainv[i * U + j] * G[j * U + i];",
     "s += Ainv[j * U + i] * G[j * U + i];"),
    ("exact SINR taken as mu", "rho[i] = mu[i] / (1.0 - mu[i]);", "rho[i] = mu[i];"),
    ("exact LLR point ignores the gain", "zi / (mu[i] * sqrt(Es))", "zi / sqrt(Es)"),
    # fixed-point datapath (Section IV-C)
    ("fixed: p z dropped", "dinv[u] * ire + (p[u] * z[2 * u] << 11)", "dinv[u] * ire"),
    ("fixed: inner product without the conjugate", "ire += hr * r[2 * i] + hi * r[2 * i + 1];",
     "ire += hr * r[2 * i] - hi * r[2 * i + 1];"),
    ("fixed: table at interval starts", "((double)idx + 0.5) / 2048.0", "((double)idx) / 2048.0"),
    ("fixed: 10-bit table index", "(x >> (n - 12)) & 2047", "(x >> (n - 11)) & 1023"),
    ("fixed: truncation instead of rounding", "return (v + ((int64_t)1 << (s - 1))) >> s;",
     "return v >> s;"),
    ("fixed: no saturation", "return v < -32768 ? -32768 : (v > 32767 ? 32767 : v);", "return v;"),
    ("fixed: residual update sign", "r[2 * i] = fx_sat16(r[2 * i] - fx_round_shift(",
     "r[2 * i] = fx_sat16(r[2 * i] + fx_round_shift("),
    ("fixed: one-sided clip", "if (cre < -beta_fx) cre = -beta_fx;", ""),
    ("fixed: p without the shift", "fx_round_shift(dinv[u] * (g >> b), 22)",
     "fx_round_shift(dinv[u] * g, 22)"),
]

BATTERY = [
    lambda: pins.test_ocd_equals_plain_cd("mmse", 32, 8, 3, 4),
    lambda: pins.test_ocd_equals_plain_cd("box", 16, 5, 4, 6),
    lambda: pins.test_ocd_equals_plain_cd("hybrid", 32, 8, 3, 4),
    lambda: pins.test_mmse_ocd_converges_to_cholesky_solution(32, 8),
    lambda: pins.test_box_ocd_converges_to_bruteforce_box_qp(3, 0.0),
    lambda: pins.test_objective_never_increases("box"),
    lambda: pins.test_single_user_closed_form("mmse"),
    lambda: pins.test_single_user_closed_form("box"),
    lambda: pins.test_paper_qpsk_box_example(),
    lambda: pins.test_default_box_is_constellation_edge(),
    lambda: pins.test_orthogonal_columns_match_exact_mmse_soft_output(6),
    lambda: pins.test_llr_2d_bruteforce_equals_per_axis(4, "box"),
    lambda: pins.test_llr_sign_equals_sliced_bits(6, "mmse"),
    lambda: pins.test_high_snr_recovers_transmitted_bits(6, "mmse"),
    lambda: pins.test_constellation_gray_neighbours_differ_in_one_bit(),
    lambda: pins.test_symbol_energy_is_a_pure_scale("mmse"),
    lambda: pins.test_symbol_energy_is_a_pure_scale("box"),
    lambda: pins.test_reference_gradient_matches_finite_differences("hybrid"),
    lambda: pins.test_reference_gradient_matches_finite_differences("box"),
    lambda: mpins.test_mmse_satisfies_the_normal_equations(32, 8, 2.5),
    lambda: mpins.test_mmse_matches_a_library_solve(),
    lambda: mpins.test_mmse_is_the_limit_of_coordinate_descent(),
    lambda: mpins.test_gain_and_sinr_are_those_of_the_error_covariance(3.0),
    lambda: mpins.test_single_user_closed_form(4),
    lambda: mpins.test_orthogonal_columns_equal_one_ocd_sweep(6),
    lambda: mpins.test_high_snr_llr_signs_are_the_transmitted_bits(),
    lambda: fpins.test_reciprocal_unit_error_bound(22),
    lambda: fpins.test_exact_orthogonal_channels_recover_the_symbols("mmse", 3),
    lambda: fpins.test_exact_orthogonal_channels_recover_the_symbols("box", 3),
    lambda: fpins.test_close_to_the_floating_point_oracle(100, 6, "mmse"),
    lambda: fpins.test_close_to_the_floating_point_oracle(128, 8, "box"),
    lambda: fpins.test_rounding_is_unbiased(),
    lambda: fpins.test_saturation_and_box_clip_closed_form(),
]


@pytest.fixture
def swap_oracle():
    saved = oracle._lib
    yield
    oracle._lib = saved


def _compile(src_text, tmp_path):
    c = tmp_path / "mut.c"
    so = tmp_path / "libmut.so"
    c.write_text(src_text)
    subprocess.check_call(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
                           "-shared", str(c), "-o", str(so), "-lm"])
    return str(so)


def test_unmutated_copy_passes_every_pin(tmp_path, swap_oracle):
    oracle._lib = oracle._open(_compile(open(SRC).read(), tmp_path))
    for check in BATTERY:
        check()


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(name, old, new, tmp_path, swap_oracle):
    text = open(SRC).read()
    assert old in text, "mutation site not found: the oracle changed, update the mutant"
    oracle._lib = oracle._open(_compile(text.replace(old, new), tmp_path))
    failures = 0
    for check in BATTERY:
        try:
            check()
        except (AssertionError, ValueError, IndexError, FloatingPointError):
            failures += 1
    assert failures > 0, "no pin caught the mutant: " + name
