"""Planted mistakes in the oracle (on the CPU) must each fail at least one pin.

Each mutation patches one function of the oracle module the way a plausible
transcription error would (a dropped term, a wrong sign or index, a transposed
operand, a wrong factor), runs the whole pin suite, and restores the module.
"""
import numpy as np
import pytest

from oracle import mcpt_oracle as M
from . import pins


def _drop_x_coupling(V, T_x, T_y, D):
    return D * (V + np.einsum("iaJB,jJbB->iajb", V, M.spin_adapted(T_y)))


def _drop_y_coupling(V, T_x, T_y, D):
    return D * (V + np.einsum("IAjb,iIaA->iajb", V, M.spin_adapted(T_x)))


def _wrong_swap(T):
    return 2.0 * T - T.transpose(0, 1, 3, 2)


def _one_sided_pair_term(V, Tau):
    return 2.0 * np.einsum("IAkc,iakc->iIaA", V, Tau)


def _printed_half_pair_term(V, Tau):
    # the pair term of Eq. 58 as printed, without the sum over the spins of k, c
    return np.einsum("IAkc,iakc->iIaA", V, Tau) + np.einsum("iakc,IAkc->iIaA", V, Tau)


def _transposed_x_coupling(V, T_x, T_y, D):
    from_x = np.einsum("IAjb,IiAa->iajb", V, M.spin_adapted(T_x))
    from_y = np.einsum("iaJB,jJbB->iajb", V, M.spin_adapted(T_y))
    return D * (V + from_x + from_y)


def _ed2_factor_two(V, Tau):
    return 2.0 * float(np.einsum("iajb,iajb->", V, Tau))


def _em2_exchange_sign(K, T):
    return float(np.einsum("ijab,ijab->", 2.0 * K + K.transpose(1, 0, 2, 3), T))


def _coupling_sign(K, D_x, couplings):
    rhs = K.copy()
    for c in couplings:
        rhs = rhs - c
    return D_x * rhs


def _literal_sign(K, D_x, couplings):
    rhs = K.copy()
    for c in couplings:
        rhs = rhs + c
    return -D_x * rhs


def _pair_denominator_swapped(ex_occ, ex_vir, ey_occ, ey_vir):
    return M.__dict__["_orig_pair_denominator"](ex_occ, ey_vir, ey_occ, ex_vir) \
        if ex_vir.shape == ey_vir.shape else 1.0 / (
            ex_occ[:, None, None, None] - ex_vir[None, :, None, None]
            + ey_occ[None, None, :, None] - ey_vir[None, None, None, :] - 1e-3)


def _monomer_denominator_wrong(e_occ, e_vir):
    return 1.0 / (e_occ[:, None, None, None] - e_occ[None, :, None, None]
                  - e_vir[None, None, :, None] - e_vir[None, None, None, :])


def _monomer_phase_no_transpose(self, Tau, monomers=None):
    monomers = range(self.N) if monomers is None else monomers
    out = []
    for x in monomers:
        cs = []
        for p, first in self.nb[x]:
            V = self.V(p)
            if first:
                cs.append(M.pair_coupling(V, Tau[p]))
            else:
                cs.append(M.pair_coupling(V.transpose(2, 3, 0, 1), Tau[p]))
        out.append(M.monomer_amplitudes(self.K[x], self.D[x], cs))
    return out


def _first_order_literal(self):
    return [self.K[x].copy() for x in range(self.N)]


MUTATIONS = {
    "drop T_X coupling of Eq. 59": ("dimer_amplitudes", _drop_x_coupling),
    "drop T_Y coupling of Eq. 59": ("dimer_amplitudes", _drop_y_coupling),
    "virtual instead of occupied swap in 2T - T": ("spin_adapted", _wrong_swap),
    "transposed T_X in Eq. 59": ("dimer_amplitudes", _transposed_x_coupling),
    "one-sided pair term of Eq. 58": ("pair_coupling", _one_sided_pair_term),
    "printed pair term of Eq. 58 without its spin sum": ("pair_coupling", _printed_half_pair_term),
    "factor 2 in Eq. 55": ("dimer_energy", _ed2_factor_two),
    "exchange sign in Eq. 54": ("monomer_energy", _em2_exchange_sign),
    "coupling sign opposite to source in Eq. 58": ("monomer_amplitudes", _coupling_sign),
    "literal sign reading of Eq. 58": ("monomer_amplitudes", _literal_sign),
    "pair denominator with swapped virtuals": ("pair_denominator", _pair_denominator_swapped),
    "monomer denominator with a sign error": ("monomer_denominator", _monomer_denominator_wrong),
    "reversed pair used untransposed": ("Oracle.monomer_phase", _monomer_phase_no_transpose),
    "integrals themselves as initial guess": ("Oracle.first_order", _first_order_literal),
}


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_mutation_is_caught(name, monkeypatch):
    target, fn = MUTATIONS[name]
    monkeypatch.setitem(M.__dict__, "_orig_pair_denominator", M.pair_denominator)
    if target.startswith("Oracle."):
        monkeypatch.setattr(M.Oracle, target.split(".")[1], fn)
    else:
        monkeypatch.setattr(M, target, fn)
    failed = [p.__name__ for p in pins.ALL_PINS if not p(M)[0]]
    assert failed, f"no pin caught the mutation '{name}'"
