"""The batched workload recipe (host only): 16 cubic cells with a ~ U{8..16}
bohr, E_cut 12 Ha, k ~ U[0, 0.5)^3, grid n = smallest {2,3,5}-smooth >= 3a,
1-8 atoms and nband in {32, 64, 128, 256}; plane-wave counts between 1000 and
8200 (the sphere of radius sqrt(2 E_cut) a / (2 pi) holds about 1000 points at
a = 8 and 8200 at a = 16)."""
import numpy as np

import workloads as W
from oracle.sphere import gsphere


def test_smooth_235():
    assert [W.smooth_235(m) for m in (1, 7, 11, 24, 26, 28, 31, 33, 44, 46, 49)] == \
        [1, 8, 12, 24, 27, 30, 32, 36, 45, 48, 50]


def test_batch_recipe():
    bs = W.make_batch()
    assert len(bs) == W.BATCH["nsys"] == 16
    for s in bs:
        assert 8 <= s.a <= 16 and float(s.a).is_integer()
        assert s.ngrid == (W.smooth_235(int(3 * s.a)),) * 3
        assert 1 <= s.natom <= 8 and s.nband in (32, 64, 128, 256)
        assert np.all((0.0 <= s.kpt_red) & (s.kpt_red < 0.5))
        assert s.ecut == 12.0 and s.degree == 8
        npw = gsphere(s.lattice, s.kpt_red, s.ecut, s.ngrid).npw
        assert 1000 <= npw <= 8200
    # seeded: the same draw twice
    again = W.make_batch()
    for s, t in zip(bs, again):
        assert s.a == t.a and np.array_equal(s.tau, t.tau) and np.array_equal(s.dij, t.dij)
    # uneven sizes: more than one grid and more than one band count
    assert len({s.ngrid for s in bs}) > 2 and len({s.nband for s in bs}) > 2
