"""The library's optimal domain-wall weights (dwf_odwf_weights, host code: an
elliptic-function closed form with its own arithmetic-geometric-mean
evaluation) against the oracle's (a Remez exchange on the minimax definition,
pinned in the oracle's pins), and the library's own error cases.  CPU only."""
import numpy as np
import pytest


@pytest.mark.parametrize("ns,a,b", [(1, 0.1, 2.0), (4, 0.05, 6.0), (8, 0.3, 4.0), (16, 0.01, 7.0), (32, 0.02, 5.0),
                                    (12, 0.999, 1.0)])
def test_weights_match_oracle(ns, a, b):
    import paper_1101_0423_amd as dwf
    from oracle import zolotarev
    w = dwf.odwf_weights(ns, a, b)
    wo = zolotarev.optimal_omega(ns, a, b)
    assert np.all(np.diff(w) <= 0)                      # largest first, as the oracle orders them
    assert np.max(np.abs(w - wo) / wo) < 1e-11, (w, wo)


def test_degenerate_interval_and_errors():
    import paper_1101_0423_amd as dwf
    assert np.allclose(dwf.odwf_weights(6, 0.7, 0.7), 1 / 0.7, rtol=1e-15, atol=0)
    for args in [(0, 0.1, 1.0), (4, 0.0, 1.0), (4, 1.0, 0.5), (4, -1.0, 1.0), (4, 0.1, np.inf)]:
        with pytest.raises(dwf.DwfError) as ei:
            dwf.odwf_weights(*args)
        assert ei.value.code == dwf.DWF_EINVAL
