"""Pins of the paper's scheme algebra (Secs. 2-5, Table 1), on the CPU.

The model in scheme_model.py is written from the step matrices the paper
prints; these tests check (i) that every scheme composes to the polyphase
matrix N_{P,U} (the paper's correctness claim for Monolithic in Sec. 3 and
for all schemes in the Conclusions), (ii) that operation and barrier counts
reproduce Table 1 (golden file transcribed from the paper), and (iii) the
inverse factorisation used by the GPU inverse kernels.
"""
import os

import pytest
import sympy as sp

import scheme_model as sm

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE1 = sm.read_table1(os.path.join(HERE, "golden", "table1_barriers_operations.txt"))
WAV = sm.paper_wavelets()


def _N(pairs):
    return sm.product([sm.N_PU(sm.sub(P, sm.zm), sm.sub(U, sm.zm), sm.sub(P, sm.zn),
                                sm.sub(U, sm.zn)) for P, U in pairs])


def test_wavelet_definitions_match_golden():
    """The model's 5/3 and DD 13/7 operators are the ones printed in Sec. 5."""
    terms = sm.read_wavelet_terms(os.path.join(HERE, "golden", "wavelet_definitions.txt"))
    for wav in ("cdf53", "dd137"):
        P, U = WAV[wav][0]
        assert sp.expand(P - sm.poly_from_terms(terms[(wav, "P")])) == 0
        assert sp.expand(U - sm.poly_from_terms(terms[(wav, "U")])) == 0


@pytest.mark.parametrize("wav", ["cdf53", "cdf97", "dd137"])
@pytest.mark.parametrize("scheme", sm.LIFTING_SCHEMES)
def test_scheme_composes_to_polyphase_matrix(wav, scheme):
    steps = []
    for P, U in WAV[wav]:
        steps += sm.scheme_steps(scheme, P, U)
    diff = (sm.product(steps) - _N(WAV[wav])).applyfunc(sp.expand)
    assert diff == sp.zeros(4, 4)


@pytest.mark.parametrize("wav", ["cdf53", "cdf97", "dd137"])
@pytest.mark.parametrize("scheme", sm.LIFTING_SCHEMES)
def test_table1_operations_and_barriers(wav, scheme):
    steps = []
    for P, U in WAV[wav]:
        steps += sm.scheme_steps(scheme, P, U)
    assert (sm.barriers(steps), sm.operations(steps)) == TABLE1[(wav, scheme)]


@pytest.mark.parametrize("wav", ["cdf53", "cdf97", "dd137"])
def test_table1_convolution(wav):
    """The Convolution scheme: four 2-D filters, one initial barrier.  Operations
    are the non-zero taps of the four filters: for DD 13/7 the 13-tap low-pass
    has 11 non-zero taps and the 7-tap high-pass 5, so 11*11 + 2*11*5 + 5*5 = 256,
    as printed (the printed cell is not a copy of the 9/7 value)."""
    bar, ops = TABLE1[(wav, "convolution")]
    assert bar == 1
    assert sm.convolution_operations(WAV[wav]) == ops


def test_dd137_filter_lengths():
    P, U = WAV["dd137"][0]
    V = sp.expand(P * U + 1)
    # low-pass = [V, U] in polyphase: 7 even + 4 odd non-zero taps; high-pass = [P, 1]
    assert sm.count_terms(V.subs(sm.z, sm.zm)) == 7
    assert sm.count_terms(U.subs(sm.z, sm.zm)) == 4
    assert sm.count_terms(P.subs(sm.z, sm.zm)) == 4
    assert sm.convolution_operations(WAV["dd137"]) == 11 * 11 + 2 * 11 * 5 + 5 * 5


def test_monolithic_star_factors_commute():
    """All four predict factors of Monolithic* commute, as do all update factors,
    so the kernel may apply the local (P0, U0) parts before or after the
    neighbour part (Sec. 4)."""
    P, U = WAV["cdf53"][0]
    steps = sm.scheme_steps("monolithic*", P, U)
    T1, TH0, TV0, S1, SH0, SV0 = steps
    for A, B in [(T1, TH0), (T1, TV0), (TH0, TV0), (S1, SH0), (S1, SV0), (SH0, SV0)]:
        assert ((A * B) - (B * A)).applyfunc(sp.expand) == sp.zeros(4, 4)


def test_iwahashi_star_order_matters():
    """In Iwahashi* the scalar predict parts must be applied first (Sec. 4):
    T^I_{P1} does not commute with T^H_{P0}."""
    P, U = WAV["cdf53"][0]
    T_I1 = sm.scheme_steps("iwahashi*", P, U)[2]
    TH0 = sm.scheme_steps("iwahashi*", P, U)[0]
    assert ((T_I1 * TH0) - (TH0 * T_I1)).applyfunc(sp.expand) != sp.zeros(4, 4)


def _neg(pairs):
    return [(-P, -U) for P, U in pairs]


@pytest.mark.parametrize("wav", ["cdf53", "cdf97"])
def test_inverse_monolithic_star(wav):
    """The inverse used by the GPU kernels: per pair in reverse order, the local
    update parts S^V_{-U0}, S^H_{-U0}, then S_{-U1} (one barrier), then the local
    predict parts T^V_{-P0}, T^H_{-P0}, then T_{-P1} (one barrier).  It composes
    with the forward Monolithic* transform to the identity."""
    fwd = []
    for P, U in WAV[wav]:
        fwd += sm.scheme_steps("monolithic*", P, U)
    inv = []
    for P, U in reversed(WAV[wav]):
        P0, P1 = sm.split(P)
        U0, U1 = sm.split(U)
        inv += [sm.S_V(-U0), sm.S_H(-U0), sm.S_M(-sm.sub(U1, sm.zm), -sm.sub(U1, sm.zn)),
                sm.T_V(-P0), sm.T_H(-P0), sm.T_M(-sm.sub(P1, sm.zm), -sm.sub(P1, sm.zn))]
    assert sm.product(fwd + inv) == sp.eye(4)
    assert sm.barriers(inv) == sm.barriers(fwd)


@pytest.mark.parametrize("scheme", ["sweldens", "iwahashi"])
def test_inverse_baselines(scheme):
    """Inverse of the separable and Iwahashi schemes: each step's matrix with the
    operators negated undoes it, except the Iwahashi spatial steps whose
    inverses are given explicitly here."""
    P, U = WAV["cdf53"][0]
    fwd = sm.scheme_steps(scheme, P, U)
    inv = [F.inv().applyfunc(sp.expand) for F in reversed(fwd)]
    assert sm.product(fwd + inv) == sp.eye(4)
    # Each inverse step reads the same neighbours as its forward step.
    assert sm.barriers(inv) == sm.barriers(fwd)
