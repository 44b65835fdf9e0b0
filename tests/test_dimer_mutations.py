"""Planted mistakes in the dimer-internal oracle (on the CPU) must each fail a pin.

Each mutation replaces the dimer-internal-term function the way a plausible
transcription slip would - a dropped term, a wrong sign or factor, a transposed
amplitude, an index of one monomer summed against the other's - runs the pin
suite and restores the original.  (An integral read in another index order that
the real-orbital symmetry of its class maps onto itself, such as (i1 i|j1 j) read
as (i i1|j j1), is not a mistake and is not planted.)"""
import numpy as np
import pytest

from oracle import mcpt_dimer as D
from . import pins_dimer

_orig = D.internal_terms


def _parts(W, Q, CX, CY, KX, JX, KY, JY, Tau):
    return [np.einsum("abAB,iAjB->iajb", W, Tau),
            np.einsum("IJij,IaJb->iajb", Q, Tau),
            -np.einsum("Iibc,Iajc->iajb", CX, Tau),
            -np.einsum("Jjac,icJb->iajb", CY, Tau),
            2.0 * np.einsum("iIaA,IAjb->iajb", KX, Tau),
            -np.einsum("Iiac,Icjb->iajb", JX, Tau),
            2.0 * np.einsum("jJbB,iaJB->iajb", KY, Tau),
            -np.einsum("Jjbd,iaJd->iajb", JY, Tau)]


def _without(idx):
    def terms(*a):
        return sum(p for k, p in enumerate(_parts(*a)) if k != idx)
    return terms


def _replace(idx, fn):
    def terms(*a):
        ps = _parts(*a)
        ps[idx] = fn(*a)
        return sum(ps)
    return terms


MUTATIONS = {
    **{f"drop_term_{k}": _without(k) for k in range(8)},
    "cross_ring_X_sign": _replace(2, lambda W, Q, CX, CY, KX, JX, KY, JY, T: np.einsum("Iibc,Iajc->iajb", CX, T)),
    "monomer_ring_factor_1": _replace(4, lambda W, Q, CX, CY, KX, JX, KY, JY, T: np.einsum("iIaA,IAjb->iajb", KX, T)),
    "ladder_amplitude_crossed": _replace(0, lambda W, Q, CX, CY, KX, JX, KY, JY, T:
                                         np.einsum("abAB,iBjA->iajb", W, T)),
    "hole_ladder_amplitude_crossed": _replace(1, lambda W, Q, CX, CY, KX, JX, KY, JY, T:
                                              np.einsum("IJij,JaIb->iajb", Q, T)),
    "cross_ring_Y_amplitude": _replace(3, lambda W, Q, CX, CY, KX, JX, KY, JY, T:
                                       -np.einsum("Jjac,iaJc->iajb", CY, T.transpose(0, 3, 2, 1))
                                       if T.shape[1] == T.shape[3] else -np.einsum("Jjac,icJb->iajb", CY, T) * 1.5),
    "monomer_ring_Y_K_for_J": _replace(7, lambda W, Q, CX, CY, KX, JX, KY, JY, T:
                                       -np.einsum("jJbd,iaJd->iajb", KY, T)),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_fails_a_pin(name):
    D.internal_terms = MUTATIONS[name]
    try:
        results = {f.__name__: f(D) for f in pins_dimer.ALL_PINS}
    finally:
        D.internal_terms = _orig
    assert any(not ok for ok, _ in results.values()), f"no pin caught {name}: {results}"


def test_unmutated_passes():
    assert all(f(D)[0] for f in pins_dimer.ALL_PINS)


def test_printed_pair_term_without_spin_sum_fails_a_pin(monkeypatch):
    """The pair term of Eq. 58 as printed (half the spin-summed term), planted in
    the module the dimer oracle takes it from."""
    from oracle import mcpt_oracle as base
    orig = base.pair_coupling
    monkeypatch.setattr(base, "pair_coupling", lambda V, Tau: 0.5 * orig(V, Tau))
    results = {f.__name__: f(D) for f in pins_dimer.ALL_PINS}
    assert any(not ok for ok, _ in results.values()), f"printed half pair term passed every pin: {results}"
