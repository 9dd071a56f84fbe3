"""The largest lattice the library takes (nx * ny = 2^28 sites, 36.5 GB of
device state), checked by an exact symmetry rather than against the oracle
(which cannot run at that size).

A periodic 16384 x 16384 lattice whose potential and initial state repeat a
64 x 64 pattern evolves into the same repetition of the 64 x 64 lattice's
own evolution: the flow commutes with lattice translations (Sec. 2.1), and
so does every part of a step here.  Each site's values are computed from its
neighbours alone, whatever the tiling of the launch, and the Newton
tolerance test takes the max norm, which is the same for the repeated
field.  So the two runs must agree bit for bit on every site, and the
64 x 64 run is itself compared with the oracle.  The energies must agree
too: the big lattice's H is 2^16 times the small one's, a power of two.
"""
import numpy as np
import pytest

import lattice_inputs as L
import oracle as O
from gpu_common import torch_cuda
from paper_2003_04345_amd import mb4 as M

pytestmark = pytest.mark.gpu

SMALL = 64
REP = 256          # 64 * 256 = 16384, 16384^2 = 2^28 sites
STEPS = 3


def test_largest_lattice_repeats_the_small_one_bit_for_bit():
    torch_cuda()
    cfg = L.config("lattice256", nx=SMALL, ny=SMALL, initial="random", seed=99,
                   defect_count=20, steps=STEPS, energy_every=0)
    v, p, q = L.make_inputs(cfg)
    with M.MB4State(SMALL, SMALL, v, cfg.g, cfg.h, eps=1e-14) as st:
        st.set_state(p, q)
        h_small = st.energy()
        assert st.step(STEPS) == M.MB4_OK, M.error_detail()
        sp, sq = st.get_state()
        it_small = st.last_stats()["newton_iters"]
        h_small_end = st.energy()
    ref, _ = O.oracle_for(cfg, v, eps=1e-14, solver="gmres").run(p + 1j * q, STEPS)
    assert np.max(np.abs(sp + 1j * sq - ref)) <= 1e-13

    big = SMALL * REP
    assert big * big == 1 << 28

    def tile(a):
        return np.tile(a.reshape(SMALL, SMALL), (REP, REP)).reshape(-1)

    with M.MB4State(big, big, tile(v), cfg.g, cfg.h, eps=1e-14) as st:
        st.set_state(tile(p), tile(q))
        h_big = st.energy()
        assert st.step(STEPS) == M.MB4_OK, M.error_detail()
        assert st.last_stats()["newton_iters"] == it_small
        bp, bq = st.get_state()
        h_big_end = st.energy()

    def repeats(bigf, smallf):
        b = bigf.reshape(REP, SMALL, REP, SMALL)
        return np.array_equal(b, np.broadcast_to(smallf.reshape(1, SMALL, 1, SMALL), b.shape))

    assert repeats(bp, sp) and repeats(bq, sq)
    for hb, hs in ((h_big, h_small), (h_big_end, h_small_end)):
        assert abs(hb - REP * REP * hs) <= 4e-16 * abs(hb)
    print(f"{big}x{big} ({big * big} sites), {STEPS} steps: every 64x64 tile equals the "
          f"64x64 run bit for bit; H {h_big_end:.17g} = 2^16 x {h_small_end:.17g}")
