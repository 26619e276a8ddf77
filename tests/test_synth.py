"""Input generators: the shared-array q-point variants equal the per-q problems."""

import numpy as np

from synth import batch_system, batch_system_qpoints


def test_batch_qpoints_share_arrays_and_match_per_q_problems():
    ps = batch_system_qpoints(21)
    assert len(ps) == 4
    for n, p in enumerate(ps):
        q = batch_system(21, n)
        assert p.iq == q.iq
        assert np.array_equal(p.gsph, q.gsph) and np.array_equal(p.gtail, q.gtail)
        assert np.array_equal(p.coef, q.coef) and np.array_equal(p.energy_eV, q.energy_eV)
        assert p.coef is ps[0].coef
