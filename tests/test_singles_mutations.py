"""Planted mistakes in the singles oracle (on the CPU) must each fail a pin.

Each mutation replaces one function of the module the way a plausible slip
would (a dropped direction of a pair, a missing transpose, a wrong sign,
factor or denominator, a wrong start), runs the pin suite and restores it."""
import numpy as np
import pytest

from oracle import mcpt_singles as S
from . import pins_singles


def _drop_reverse(prob, t):
    u = [np.zeros_like(tx) for tx in t]
    for p in range(prob.n_pair):
        x, y = (int(q) for q in prob.pairs[p])
        u[x] += np.einsum("iakc,kc->ia", np.asarray(prob.v_of(p)), t[y])
    return u


def _no_transpose(prob, t):
    u = [np.zeros_like(tx) for tx in t]
    for p in range(prob.n_pair):
        x, y = (int(q) for q in prob.pairs[p])
        V = np.asarray(prob.v_of(p))
        u[x] += np.einsum("iakc,kc->ia", V, t[y])
        # the reverse direction contracted over the wrong index pair (square blocks only)
        u[y] += np.einsum("kcia,ia->kc", V.reshape(t[y].shape + t[x].shape), t[x])
    return u


def _minus_coupling(prob, t):
    return [-u for u in S.__dict__["_orig_coupling"](prob, t)]


def _swapped_occ_vir(prob, t):
    u = [np.zeros_like(tx) for tx in t]
    for p in range(prob.n_pair):
        x, y = (int(q) for q in prob.pairs[p])
        V = np.asarray(prob.v_of(p))
        ty, tx = t[y], t[x]
        u[x] += np.einsum("iakc,kc->ia", V, ty) if ty.shape[0] != ty.shape[1] else \
            np.einsum("iakc,ck->ia", V, ty)
        u[y] += np.einsum("iakc,ia->kc", V, tx)
    return u


def _printed_half(prob, t):
    # the pair sum of Eq. 57 as printed, without the sum over the spins of k, c
    return [0.5 * u for u in S.__dict__["_orig_coupling"](prob, t)]


def _intra_factor_one(K, J, t):
    return S.__dict__["_orig_intramonomer"](0.5 * K, J, t)


def _intra_exchange_sign(K, J, t):
    return S.__dict__["_orig_intramonomer"](K, -J, t)


def _intra_classes_swapped(K, J, t):
    return S.__dict__["_orig_intramonomer"](J, K, t)


def _energy_factor_one(w, t):
    return float(np.sum(w * t))


def _denominator_reversed(e_occ, e_vir):
    return 1.0 / (e_vir[None, :] - e_occ[:, None])


MUTATIONS = {
    "drop_reverse_direction": ("coupling", _drop_reverse),
    "reverse_without_transpose": ("coupling", _no_transpose),
    "coupling_sign": ("coupling", _minus_coupling),
    "printed_pair_sum_without_spin_sum": ("coupling", _printed_half),
    "intramonomer_direct_factor_one": ("intramonomer", _intra_factor_one),
    "intramonomer_exchange_sign": ("intramonomer", _intra_exchange_sign),
    "intramonomer_k_and_j_swapped": ("intramonomer", _intra_classes_swapped),
    "occ_vir_swapped_in_t": ("coupling", _swapped_occ_vir),
    "energy_factor_one": ("singles_energy", _energy_factor_one),
    "denominator_reversed": ("singles_denominator", _denominator_reversed),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_fails_a_pin(name):
    attr, fn = MUTATIONS[name]
    orig = getattr(S, attr)
    S.__dict__["_orig_" + attr] = orig
    setattr(S, attr, fn)
    try:
        results = {p.__name__: p(S) for p in pins_singles.ALL_SINGLES_PINS}
    finally:
        setattr(S, attr, orig)
    failed = [k for k, (ok, _) in results.items() if not ok]
    assert failed, f"mutation {name} passed every pin"
