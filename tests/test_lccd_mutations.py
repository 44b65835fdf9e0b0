"""Planted mistakes in the full-monomer-equation oracle (on the CPU) must each
fail a pin.

Each mutation replaces the intramonomer-term function (or the integral naming)
the way a plausible transcription slip would - a dropped term, a wrong sign, an
index swap in T, the K and J classes exchanged, a missing transpose - runs the
pin suite and restores the original."""
import numpy as np
import pytest

from oracle import mcpt_lccd as L
from . import pins_lccd

_orig_terms = L.intramonomer_terms
_orig_named = L.named_integrals


def _without(idx):
    """The printed terms with term idx (0-based, in printed order) left out."""
    def terms(v, T):
        ring = v["voov"] - v["vovo"].transpose(0, 1, 3, 2)
        T_ex = T - T.transpose(1, 0, 2, 3)
        parts = [np.einsum("abcd,ijcd->ijab", v["vvvv"], T),
                 np.einsum("klij,klab->ijab", v["oooo"], T),
                 np.einsum("akic,kjcb->ijab", ring, T),
                 np.einsum("bkjc,kica->ijab", ring, T),
                 np.einsum("kaci,kjcb->ijab", v["ovvo"], T_ex),
                 np.einsum("kbcj,kica->ijab", v["ovvo"], T_ex),
                 -np.einsum("bkci,kjac->ijab", v["vovo"], T),
                 -np.einsum("akcj,kibc->ijab", v["vovo"], T)]
        return sum(p for k, p in enumerate(parts) if k != idx)
    return terms


def _ring_sign(v, T):
    # the exchange part of the first ring combination added instead of subtracted
    ring_bad = v["voov"] + v["vovo"].transpose(0, 1, 3, 2)
    return _orig_terms(v, T) + np.einsum("akic,kjcb->ijab", ring_bad - (v["voov"] - v["vovo"].transpose(0, 1, 3, 2)), T)


def _ladder_transposed(v, T):
    # T^{a2 a3} read as T^{a3 a2} in the particle-particle ladder
    good = np.einsum("abcd,ijcd->ijab", v["vvvv"], T)
    bad = np.einsum("abcd,ijdc->ijab", v["vvvv"], T)
    return _orig_terms(v, T) - good + bad


def _hole_ladder_swapped(v, T):
    # v^{i2 i3}_{i i1} read as v^{i i1}_{i2 i3}
    good = np.einsum("klij,klab->ijab", v["oooo"], T)
    bad = np.einsum("ijkl,klab->ijab", v["oooo"], T)
    return _orig_terms(v, T) - good + bad


def _exchange_T_wrong(v, T):
    # T^{a2 a1}_{i1 i2} taken as T^{a1 a2}_{i1 i2}
    good = np.einsum("kaci,kjcb->ijab", v["ovvo"], T - T.transpose(1, 0, 2, 3))
    bad = np.einsum("kaci,kjcb->ijab", v["ovvo"], T - T.transpose(1, 0, 3, 2))
    return _orig_terms(v, T) - good + bad


def _k_for_j(K, J, W, Q):
    # the (oo|vv) class replaced by the (ov|ov) one
    return _orig_named(K, K, W, Q)


def _j_untransposed(K, J, W, Q):
    # J read as J[i, k, a, c] instead of J[k, i, a, c]
    out = _orig_named(K, J, W, Q)
    out["vovo"] = J.transpose(1, 0, 2, 3).transpose(2, 0, 3, 1)
    return out


MUTATIONS = {f"drop_term_{k + 1}": ("intramonomer_terms", _without(k)) for k in range(8)}
MUTATIONS.update({
    "ring_exchange_sign": ("intramonomer_terms", _ring_sign),
    "pp_ladder_transposed": ("intramonomer_terms", _ladder_transposed),
    "hh_ladder_swapped": ("intramonomer_terms", _hole_ladder_swapped),
    "exchange_amplitude_wrong_swap": ("intramonomer_terms", _exchange_T_wrong),
    "k_class_for_j": ("named_integrals", _k_for_j),
    "j_occupied_swapped": ("named_integrals", _j_untransposed),
})


def first_failing_pin():
    """Name of the first pin (in suite order) the oracle as it stands fails, or None."""
    for p in pins_lccd.ALL_LCCD_PINS:
        if not p(L)[0]:
            return p.__name__
    return None


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_fails_a_pin(name):
    attr, fn = MUTATIONS[name]
    orig = getattr(L, attr)
    setattr(L, attr, fn)
    try:
        failed = first_failing_pin()
    finally:
        setattr(L, attr, orig)
    assert failed, f"mutation {name} passed every pin"


def test_printed_pair_term_without_spin_sum_fails_a_pin(monkeypatch):
    """The pair term of Eq. 58 as printed (half the spin-summed term), planted in
    the module the full-equation oracle takes it from."""
    from oracle import mcpt_oracle as base
    orig = base.pair_coupling
    monkeypatch.setattr(base, "pair_coupling", lambda V, Tau: 0.5 * orig(V, Tau))
    assert first_failing_pin(), "printed half pair term passed every pin"
