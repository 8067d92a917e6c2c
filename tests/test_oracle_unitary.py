"""Pins of the oracle's random unitary circulant (Section 6, Example exunc).

Example exunc builds the multiplier from a spectrum u of unit-modulus entries
with random phases and takes its first column c = Omega^{-1} u, where Omega
is the DFT matrix (w^{jk}), w = exp(2 pi i / n).  This project reads it for
real matrices: u conjugate-symmetric (u_{n-j} = conj(u_j)), u_0 and, for even
n, u_{n/2} equal to +1 or -1.  What the mathematics fixes, checked here
independently of the oracle's own arithmetic:
* Theorem thcpw: C = Omega^{-1} diag(u) Omega, so Omega c = u; numpy's FFT
  (a library routine) of the oracle's c must return the oracle's u;
* |u_j| = 1 makes C orthogonal: C C^T = I;
* small sizes worked by hand: n = 1, 2 from the signs, n = 4 in closed form
  c_k = (u_0 + (-1)^k u_2 + 2 cos(2 pi phi_1 - pi k / 2)) / 4;
* the phases are the stream-4 uniforms of the written RNG specification;
* the first column is real (the imaginary parts cancel);
* the method's invariant: the singular-leading-block input that breaks plain
  GENP is solved after preprocessing, eta <= 1e-13 after one refinement step.
Plausible slips each break one of these: the opposite sign of the exponent
(n = 4 closed form, FFT), a missing 1/n (orthogonality), a spectrum that is
not conjugate-symmetric (real column), phases from another stream.
"""
import numpy as np
import pytest

import oracle
import workloads

EPS = np.finfo(np.float64).eps
U = oracle.UNITARY_CIRCULANT


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 63, 64, 257, 1000])
def test_spectrum_unit_modulus_conjugate_symmetric(orc, n):
    u = oracle.unitary_spectrum(n, seed=11 + n)
    assert np.allclose(np.abs(u), 1.0, rtol=0, atol=4 * EPS)
    j = np.arange(1, n)
    assert np.array_equal(u[n - j], np.conj(u[j]))
    assert u[0].imag == 0 and abs(u[0].real) == 1.0
    if n % 2 == 0:
        assert u[n // 2].imag == 0 and abs(u[n // 2].real) == 1.0


@pytest.mark.parametrize("n", [3, 8, 100, 1001])
def test_phases_are_stream4_uniforms(orc, n):
    seed = 77
    phi = oracle.uniforms(seed, 4, n)
    u = oracle.unitary_spectrum(n, seed)
    for j in range(1, (n + 1) // 2):
        assert abs(u[j] - np.exp(2j * np.pi * phi[j])) <= 4 * EPS
    assert u[0].real == (1.0 if phi[0] < 0.5 else -1.0)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 16, 255, 1024])
def test_theorem_thcpw_fft_of_column_returns_spectrum(orc, n):
    seed = 5 + n
    u = oracle.unitary_spectrum(n, seed)
    c = oracle.multiplier_params(U, n, seed)
    # Omega c with w = exp(+2 pi i / n) is n * ifft(c) in numpy's sign convention
    u_fft = n * np.fft.ifft(c)
    assert np.abs(u_fft - u).max() <= 8 * np.log2(n + 1) * EPS * np.sqrt(n) + 4 * EPS


@pytest.mark.parametrize("n", [2, 5, 64, 300, 1024])
def test_column_is_real_and_matrix_orthogonal(orc, n):
    u = oracle.unitary_spectrum(n, seed=3)
    c, imag = oracle.unitary_column(u)
    assert imag <= 8 * EPS
    C = oracle.multiplier_dense(U, n, c)
    err = np.abs(C @ C.T - np.eye(n)).max()
    assert err <= 4 * n * EPS, err
    assert np.abs(C.T @ C - np.eye(n)).max() <= 4 * n * EPS


def test_small_sizes_by_hand(orc):
    seed = 123
    # n = 1: u = (+-1), c = u
    phi = oracle.uniforms(seed, 4, 1)
    assert oracle.multiplier_params(U, 1, seed)[0] == (1.0 if phi[0] < 0.5 else -1.0)
    # n = 2: u = (s0, s1) real, c = ((s0 + s1) / 2, (s0 - s1) / 2)
    phi = oracle.uniforms(seed, 4, 2)
    s0, s1 = (1.0 if p < 0.5 else -1.0 for p in phi)
    assert np.array_equal(oracle.multiplier_params(U, 2, seed), [(s0 + s1) / 2, (s0 - s1) / 2])
    # n = 4: u = (s0, e^{i t}, s2, e^{-i t}), t = 2 pi phi_1:
    # c_k = (s0 + (-1)^k s2 + 2 cos(t - pi k / 2)) / 4
    phi = oracle.uniforms(seed, 4, 4)
    s0 = 1.0 if phi[0] < 0.5 else -1.0
    s2 = 1.0 if phi[2] < 0.5 else -1.0
    t = 2 * np.pi * phi[1]
    want = [(s0 + (-1) ** k * s2 + 2 * np.cos(t - np.pi * k / 2)) / 4 for k in range(4)]
    got = oracle.multiplier_params(U, 4, seed)
    assert np.abs(got - want).max() <= 8 * EPS
    # and it is not the transposed circulant (the other sign of the exponent)
    wrong = [(s0 + (-1) ** k * s2 + 2 * np.cos(t + np.pi * k / 2)) / 4 for k in range(4)]
    assert np.abs(got - np.asarray(wrong)).max() > 1e-3 or abs(np.sin(t)) < 1e-3


@pytest.mark.parametrize("n", [6, 31, 64])
def test_column_matches_the_dense_inverse_dft(orc, n):
    u = oracle.unitary_spectrum(n, seed=9)
    jk = np.outer(np.arange(n), np.arange(n))
    omega = np.exp(2j * np.pi * jk / n)
    c_ref = (omega.conj().T @ u) / n  # Omega^{-1} = Omega^H / n
    c, _ = oracle.unitary_column(u)
    assert np.abs(c_ref.imag).max() <= 16 * n * EPS
    assert np.abs(c - c_ref.real).max() <= 16 * n * EPS


def test_breakdown_input_solved_after_unitary_preprocessing(orc):
    A = workloads.breakdown_case(seed=0)
    b = workloads.rhs(256, 1, seed=0)
    plain = oracle.factor(A, oracle.NONE, 0)
    assert plain.status == oracle.ZERO_PIVOT and plain.info == 63
    f = oracle.factor(A, U, 1000)
    assert f.status == oracle.OK
    s = oracle.solve(f, b, refine=1)
    assert s.eta[-1] <= 1e-13
    assert np.linalg.norm(s.X - np.linalg.solve(A, b)) / np.linalg.norm(np.linalg.solve(A, b)) \
        <= 2 * np.linalg.cond(A) * 1e-13


# ---- planted slips in a compiled copy of the oracle: each must break a pin ----

import ctypes  # noqa: E402
import os  # noqa: E402
import subprocess  # noqa: E402

_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                    "rmge_oracle.c")

MUTATIONS = {
    "exponent_sign": ("const double ang = -two_pi * (double)t / (double)n;",
                      "const double ang = two_pi * (double)t / (double)n;"),
    "no_conjugate_symmetry": ("uim[n - j] = -uim[j];", "uim[n - j] = uim[j];"),
    "missing_one_over_n": ("c[k] = sre / (double)n;", "c[k] = sre / sqrt((double)n);"),
    "phases_from_circulant_stream": (
        "orc_uniforms(seed, (uint64_t)ORC_UNITARY_CIRCULANT, n, phi);",
        "orc_uniforms(seed, (uint64_t)ORC_CIRCULANT, n, phi);"),
    "cos_sin_swapped": ("ure[j] = cos(two_pi * phi[j]);", "ure[j] = sin(two_pi * phi[j]);"),
}


def _compile(tmp_path, name, text):
    path = tmp_path / ("%s.c" % name)
    path.write_text(text)
    so = tmp_path / ("%s.so" % name)
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off", str(path),
                    "-o", str(so), "-lm"], check=True)
    L = ctypes.CDLL(str(so))
    vp = ctypes.c_void_p
    L.orc_multiplier_params.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, vp]
    L.orc_uniforms.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, vp]
    return L


def _pins_hold(L):
    def column(n, seed):
        c = np.zeros(n)
        L.orc_multiplier_params(4, n, seed, c.ctypes.data_as(ctypes.c_void_p))
        return c

    ok = True
    seed = 123
    phi = oracle.uniforms(seed, 4, 4)  # the specification's stream, from the real oracle
    s0 = 1.0 if phi[0] < 0.5 else -1.0
    s2 = 1.0 if phi[2] < 0.5 else -1.0
    t = 2 * np.pi * phi[1]
    want = np.array([(s0 + (-1) ** k * s2 + 2 * np.cos(t - np.pi * k / 2)) / 4 for k in range(4)])
    ok &= bool(np.abs(column(4, seed) - want).max() <= 8 * EPS)
    for n in (5, 64):
        c = column(n, 7)
        C = oracle.multiplier_dense(oracle.CIRCULANT, n, c)
        ok &= bool(np.abs(C @ C.T - np.eye(n)).max() <= 4 * n * EPS)
        u = n * np.fft.ifft(c)
        ok &= bool(np.abs(np.abs(u) - 1.0).max() <= 64 * EPS)
    return ok


def test_unmutated_oracle_passes_the_unitary_pins(tmp_path):
    assert _pins_hold(_compile(tmp_path, "orig", open(_SRC).read()))


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_slip_breaks_a_unitary_pin(tmp_path, name):
    old, new = MUTATIONS[name]
    src = open(_SRC).read()
    assert src.count(old) == 1, name
    assert not _pins_hold(_compile(tmp_path, name, src.replace(old, new))), name
