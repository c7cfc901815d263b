"""Host checks of the random sweep cases: the library's validation accepts
every case, and the oracle returns a Hamiltonian tour whose length is the
closed tour's length (eq. 1), recomputed here independently."""

import numpy as np

import oracle
import paper_2601_19041_amd as hac
from _sweep import sweep_cases


def _tour_length(inst, tour):
    nxt = np.roll(tour, -1)
    if inst.kind == "coords":
        d = inst.coords[tour] - inst.coords[nxt]
        return float(np.sqrt((d * d).sum(1)).sum())
    return float(inst.dist[tour, nxt].sum())


def test_sweep_cases_are_valid_and_oracle_tours_hamiltonian():
    for inst, over in sweep_cases():
        assert hac.validate(inst, **over) == hac.HAC_OK, inst.name
        st, tour, L, _ = oracle.decode(inst, **over)
        assert st == 0, inst.name
        assert np.array_equal(np.sort(tour), np.arange(inst.n)), inst.name
        assert tour[0] == 0, inst.name
        assert abs(L - _tour_length(inst, tour)) <= 1e-12 * max(L, 1.0), inst.name
