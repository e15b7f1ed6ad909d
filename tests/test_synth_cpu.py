"""The seeded input generator: reproducible, and the batch recipe it states."""
import numpy as np

import synth
from synth.configs import MIN_GAP_HA


def test_batch_systems_follow_the_recipe():
    ps = synth.batch(4, seed0=3900, cells_max=2, n_omega_range=(4, 6), n_pert_range=(2, 3), workers=1)
    again = synth.batch(4, seed0=3900, cells_max=2, n_omega_range=(4, 6), n_pert_range=(2, 3), workers=1)
    for p, q in zip(ps, again):
        assert p.name == q.name
        assert np.array_equal(p.v_grid, q.v_grid) and np.array_equal(p.psi_k, q.psi_k)
        assert np.array_equal(p.dv_miller, q.dv_miller) and np.array_equal(p.qvec, q.qvec)
    for p in ps:
        cells = tuple(int(c) for c in p.name[p.name.index("(") + 1:-1].split(","))
        n_atoms = 2 * cells[0] * cells[1] * cells[2]
        assert p.grid == tuple(24 * c for c in cells)
        assert len(p.tau) == n_atoms
        assert abs(p.n_occ - 2 * n_atoms) <= 6
        assert p.eps_k[p.n_occ] - p.eps_k[p.n_occ - 1] >= MIN_GAP_HA
        assert p.eps_kq[p.n_occ] - p.eps_kq[p.n_occ - 1] >= MIN_GAP_HA
        assert 4 <= p.n_omega <= 6 and 2 <= p.n_pert <= 3
        # the sphere fits the grid without wrapping onto itself
        m = np.abs(p.miller_kq).max(axis=0)
        assert np.all(2 * m + 1 <= np.array(p.grid))
