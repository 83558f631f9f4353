"""Executable model of the paper's 2-D lifting schemes (test-only, sympy).

Every scheme is a list of 4x4 step matrices of bivariate Laurent polynomials
acting on the quadruple vector [LL, HL, LH, HH]^T, listed in the order they are
applied (right to left in the paper's formulas).  The model checks the paper's
algebra (Secs. 2-4) independently of both the oracle and the GPU kernels.

Notation (Sec. 2): z_m is the horizontal variable and z_n the vertical one;
P = P(z_m), U = U(z_m) act along rows, P* = P(z_n), U* = U(z_n) along columns.
The split of Sec. 4 writes P = P0 + P1 and U = U0 + U1 where P0, U0 are the
z^0 (scalar) coefficients.
"""
from __future__ import annotations

from fractions import Fraction
from functools import reduce

import sympy as sp

zm, zn = sp.symbols("z_m z_n")
z = sp.Symbol("z")


def sub(poly, var):
    return sp.expand(poly.subs(z, var))


def eye():
    return sp.eye(4)


def mat(rows):
    return sp.Matrix(rows)


# --- Sweldens (Sec. 2, "Sweldens Scheme") -------------------------------------
def T_H(P):
    return mat([[1, 0, 0, 0], [P, 1, 0, 0], [0, 0, 1, 0], [0, 0, P, 1]])


def T_V(Ps):
    return mat([[1, 0, 0, 0], [0, 1, 0, 0], [Ps, 0, 1, 0], [0, Ps, 0, 1]])


def S_H(U):
    return mat([[1, U, 0, 0], [0, 1, 0, 0], [0, 0, 1, U], [0, 0, 0, 1]])


def S_V(Us):
    return mat([[1, 0, Us, 0], [0, 1, 0, Us], [0, 0, 1, 0], [0, 0, 0, 1]])


# --- Polyphase (Sec. 2, "Convolution and Polyphase Schemes") ------------------
def N_PU(P, U, Ps, Us):
    V = sp.expand(P * U + 1)
    Vs = sp.expand(Ps * Us + 1)
    return mat([[Vs * V, Vs * U, Us * V, Us * U],
                [Vs * P, Vs, Us * P, Us],
                [Ps * V, Ps * U, V, U],
                [Ps * P, Ps, P, 1]]).applyfunc(sp.expand)


# --- Iwahashi (Sec. 2, "Iwahashi Scheme") -------------------------------------
def T_I(P, Ps):
    return mat([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0], [P * Ps, Ps, P, 1]])


def R_I(P, U, Ps, Us):
    return mat([[1, 0, 0, 0], [P, 1, 0, Us], [Ps, 0, 1, U], [0, 0, 0, 1]])


def S_I(U, Us):
    return mat([[1, U, Us, -U * Us], [0, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1]])


# --- Explosive (Sec. 3, "Explosive Scheme") -----------------------------------
def T_E(P, Ps):
    return mat([[1, 0, 0, 0], [P, 1, 0, 0], [Ps, 0, 1, 0], [-P * Ps, 0, 0, 1]])


def R_E(P, U, Ps, Us):
    return mat([[1, U, Us, 0], [0, 1, 0, 0], [0, 0, 1, 0], [0, Ps, P, 1]])


def S_E(U, Us):
    return mat([[1, 0, 0, U * Us], [0, 1, 0, Us], [0, 0, 1, U], [0, 0, 0, 1]])


# --- Monolithic (Sec. 3, "Monolithic Scheme") ---------------------------------
def T_M(P, Ps):
    return mat([[1, 0, 0, 0], [P, 1, 0, 0], [Ps, 0, 1, 0], [P * Ps, Ps, P, 1]])


def S_M(U, Us):
    return mat([[1, U, Us, U * Us], [0, 1, 0, Us], [0, 0, 1, U], [0, 0, 0, 1]])


def split(poly):
    """(P0, P1): the z^0 coefficient and the remainder (Sec. 4)."""
    e = sp.expand(poly)
    p0 = e.coeff(z, 0)
    return p0, sp.expand(e - p0)


def scheme_steps(name, P, U):
    """Step matrices of one predict/update pair, in order of application."""
    Pm, Um, Pn, Un = sub(P, zm), sub(U, zm), sub(P, zn), sub(U, zn)
    P0, P1 = split(P)
    U0, U1 = split(U)
    P1m, P1n, U1m, U1n = sub(P1, zm), sub(P1, zn), sub(U1, zm), sub(U1, zn)
    if name == "sweldens":
        return [T_H(Pm), T_V(Pn), S_H(Um), S_V(Un)]
    if name == "iwahashi":
        return [T_I(Pm, Pn), R_I(Pm, Um, Pn, Un), S_I(Um, Un)]
    if name == "iwahashi*":
        return [T_H(P0), T_V(P0), T_I(P1m, P1n), R_I(P1m, U1m, P1n, U1n), S_I(U1m, U1n),
                S_H(U0), S_V(U0)]
    if name == "explosive":
        return [T_E(Pm, Pn), R_E(Pm, Um, Pn, Un), S_E(Um, Un)]
    if name == "explosive*":
        return [T_H(P0), T_V(P0), T_E(P1m, P1n), R_E(P1m, U1m, P1n, U1n), S_E(U1m, U1n),
                S_H(U0), S_V(U0)]
    if name == "monolithic":
        return [T_M(Pm, Pn), S_M(Um, Un)]
    if name == "monolithic*":
        return [T_M(P1m, P1n), T_H(P0), T_V(P0), S_M(U1m, U1n), S_H(U0), S_V(U0)]
    if name == "polyphase":
        return [N_PU(Pm, Um, Pn, Un)]
    if name == "polyphase*":
        return [T_H(P0), T_V(P0), N_PU(P1m, U1m, P1n, U1n), S_H(U0), S_V(U0)]
    raise KeyError(name)


LIFTING_SCHEMES = ["sweldens", "iwahashi", "iwahashi*", "explosive", "explosive*",
                   "monolithic", "monolithic*", "polyphase", "polyphase*"]


def product(steps):
    """Composite matrix of steps applied first-to-last: M = F_last ... F_first."""
    return reduce(lambda acc, f: (f * acc).applyfunc(sp.expand), steps, eye())


def count_terms(e) -> int:
    e = sp.expand(e)
    if e == 0:
        return 0
    poly = sp.Poly(sp.expand(e * zm ** 16 * zn ** 16), zm, zn)
    return len([c for c in poly.coeffs() if c != 0])


def is_scalar(e) -> bool:
    e = sp.expand(e)
    return not (e.has(zm) or e.has(zn))


def step_operations(F) -> int:
    """Multiply-accumulate taps of a step: monomials of every entry except unit diagonals."""
    n = 0
    for i in range(4):
        for j in range(4):
            e = sp.expand(F[i, j])
            if i == j and e == 1:
                continue
            n += count_terms(e)
    return n


def step_reads_neighbours(F) -> bool:
    return any(not is_scalar(F[i, j]) for i in range(4) for j in range(4))


def operations(steps) -> int:
    return sum(step_operations(F) for F in steps)


def barriers(steps) -> int:
    """A barrier precedes every step that reads another thread's quadruple."""
    return sum(1 for F in steps if step_reads_neighbours(F))


def convolution_operations(pairs) -> int:
    """Taps of the four 2-D filters of the whole transform (every entry of N counts)."""
    N = product([N_PU(sub(P, zm), sub(U, zm), sub(P, zn), sub(U, zn)) for P, U in pairs])
    return sum(count_terms(N[i, j]) for i in range(4) for j in range(4))


def poly_from_terms(terms):
    """Laurent polynomial in z from {exponent: Fraction}, in the paper's convention."""
    return sp.expand(sum(sp.Rational(c.numerator, c.denominator) * z ** (-k)
                         for k, c in terms.items()))


def paper_wavelets():
    """Lifting pairs of the three wavelets of Sec. 5 in the paper's convention.

    CDF 9/7 uses symbols for alpha..delta: operation and barrier counts do not
    depend on their values (no cancellation can occur between distinct symbols).
    """
    a, b, g, d = sp.symbols("alpha beta gamma delta")
    zi = z ** -1
    cdf53 = [(sp.Rational(-1, 2) * (1 + zi), sp.Rational(1, 4) * (1 + z))]
    cdf97 = [(a * (1 + zi), b * (1 + z)), (g * (1 + zi), d * (1 + z))]
    dd137 = [(sp.Rational(1, 16) * (z + z ** -2) - sp.Rational(9, 16) * (1 + zi),
              sp.Rational(9, 32) * (1 + z) - sp.Rational(1, 32) * (zi + z ** 2))]
    return {"cdf53": [tuple(map(sp.expand, p)) for p in cdf53],
            "cdf97": [tuple(map(sp.expand, p)) for p in cdf97],
            "dd137": [tuple(map(sp.expand, p)) for p in dd137]}


def read_table1(path):
    rows = {}
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            wav, scheme, bar, ops = line.split()
            rows[(wav, scheme)] = (int(bar), int(ops))
    return rows


def read_wavelet_terms(path):
    out = {}
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            wav, op, exp, coef = line.split()
            # file lists exponent e of z^e; store as {-e: c} for poly_from_terms (z^-k)
            out.setdefault((wav, op), {})[-int(exp)] = Fraction(coef)
    return out
