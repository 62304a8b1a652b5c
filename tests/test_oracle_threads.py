"""The oracle's outer layer / guide-star loops on several OpenMP threads give bitwise the results
of one thread (each iteration writes its own block and every sum keeps its order)."""
import numpy as np
import pytest

from oracle import Oracle, get_threads, set_threads
from paper_2009_00946_amd import synth


@pytest.mark.parametrize("name", ["c0_tiny", "t1_mixed", "c3_mid_lgs"])
def test_threads_do_not_change_results(name):
    cfg = synth.load_config(name)
    before = get_threads()
    outs = []
    try:
        for nt in (1, 4):
            set_threads(nt)
            O = Oracle(cfg)
            s = O.Ahat(synth.layer_screens_flat(cfg)) + O.slope_mask() * synth.slope_noise(cfg)
            z = np.zeros(O.n_coef)
            c, bp, rp, res, st = O.frame(s, z, z, z, cfg["n_iter"], True)
            x = synth.normal_vector(O.n_coef, 5)
            outs.append([O.precond(), c, bp, rp, res, O.M(x), O.At(s), O.A(x), O.Wt(x), O.W(x), O.fit(c, None, 1.0)])
    finally:
        set_threads(before)
    for a, b in zip(*outs):
        assert np.array_equal(a, b)
