"""Pins for the oracle's Boys function F_m(T) = int_0^1 t^{2m} exp(-T t^2) dt.

The paper evaluates [00|00] analytically (Section 2.2); every higher integral
rests on F_m.  The oracle's value is checked against mpmath at 40 digits
through two identities that share nothing with its series / erf code:
  F_m(T) = 1F1(m+1/2; m+3/2; -T) / (2m+1)
  F_m(T) = gamma_lower(m+1/2, T) / (2 T^{m+1/2})
plus the exact values F_m(0) = 1/(2m+1) and the downward-recursion identity.
"""
import mpmath
import numpy as np
import pytest

import oracle

T_GRID = [0.0, 1e-12, 1e-6, 0.01, 0.3, 1.0, 2.5, 7.0, 12.0, 17.9, 25.0, 29.999, 30.0, 30.001, 35.0,
          50.0, 80.0, 120.0, 200.0]


def f_hyp(m, T):
    with mpmath.workdps(40):
        return mpmath.hyp1f1(m + mpmath.mpf(1) / 2, m + mpmath.mpf(3) / 2, -mpmath.mpf(T)) / (2 * m + 1)


def f_gamma(m, T):
    with mpmath.workdps(40):
        T = mpmath.mpf(T)
        if T == 0:
            return mpmath.mpf(1) / (2 * m + 1)
        a = m + mpmath.mpf(1) / 2
        return mpmath.gammainc(a, 0, T) / (2 * T ** a)


@pytest.mark.parametrize("T", T_GRID)
def test_boys_vs_mpmath(T):
    mmax = 16
    F = oracle.boys(mmax, T)
    for m in range(mmax + 1):
        ref = f_hyp(m, T)
        assert abs(F[m] - float(ref)) <= 2e-15 * float(ref), (m, T, F[m], ref)


def test_two_identities_agree():
    # the two mpmath routes agree with each other far below double precision
    for T in [0.5, 9.0, 31.0]:
        for m in (0, 5, 13):
            a, b = f_hyp(m, T), f_gamma(m, T)
            with mpmath.workdps(40):
                assert abs(a - b) < mpmath.mpf(10) ** -35 * abs(a)


def test_boys_at_zero():
    F = oracle.boys(20, 0.0)
    assert np.allclose(F, [1.0 / (2 * m + 1) for m in range(21)], rtol=1e-15, atol=0)


def test_downward_identity():
    # (2m+1) F_m = 2T F_{m+1} + exp(-T), exactly, on both sides of the T=30 switch
    for T in [0.7, 10.0, 29.5, 30.5, 60.0]:
        F = oracle.boys(14, T)
        for m in range(14):
            lhs = (2 * m + 1) * F[m]
            rhs = 2 * T * F[m + 1] + np.exp(-T)
            assert abs(lhs - rhs) <= 4e-15 * abs(lhs)


def test_asymptotic():
    # F_m(T) -> (2m-1)!! / 2^{m+1} sqrt(pi / T^{2m+1}) for large T
    T = 400.0
    F = oracle.boys(6, T)
    df = 1.0
    for m in range(7):
        ref = df / 2 ** (m + 1) * np.sqrt(np.pi / T ** (2 * m + 1))
        assert abs(F[m] - ref) <= 1e-14 * ref
        df *= 2 * m + 1


def test_bad_arguments():
    with pytest.raises(RuntimeError):
        oracle.boys(3, -1.0)
    with pytest.raises(RuntimeError):
        oracle.boys(3, float("nan"))
