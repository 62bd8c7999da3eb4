"""The allocation-free entry point ctm_free_energy_noalloc against
ctm_free_energy (same kernels, temporaries from the library's fixed scratch):
two calls in a row on one GPU, the second on a smaller context, and the
clear error when the temporaries do not fit."""
import numpy as np
import pytest

from paper_2506_19339_amd import ctm
from synth_inputs import raw_peps

pytestmark = pytest.mark.gpu


def _both(beta, D, chi, seed, moves):
    with ctm.SplitCTM(beta, raw_peps(D, seed), chi) as c:
        c.iterate(moves)
        a = c.free_energy_noalloc()
        b = c.free_energy()
    return a, b


def test_noalloc_matches_free_energy_twice():
    for beta, D, chi, seed, moves in ((0.22, 3, 30, 0, 12), (0.2, 2, 16, 4, 20)):
        a, b = _both(beta, D, chi, seed, moves)
        for x, y in zip(a, b):
            assert abs(x - y) <= 1e-13 * abs(y), (D, chi, a, b)


def test_noalloc_rejects_what_does_not_fit():
    with ctm.SplitCTM(0.22, raw_peps(5, 0), 100) as c:
        c.iterate(2)
        with pytest.raises(ctm.CtmError) as e:
            c.free_energy_noalloc()
        assert e.value.status == ctm.CTM_ENOMEM and "scratch" in str(e.value)
        f = c.free_energy()[0]          # the context is still usable
        assert np.isfinite(f)
