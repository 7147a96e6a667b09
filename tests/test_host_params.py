"""Host-side parameter tables of the package (no GPU): the Lorentz-Berthelot mixing helper."""
import numpy as np
import pytest


def test_lorentz_berthelot_table_and_errors():
    from paper_2508_06628_amd import api
    t = api.lorentz_berthelot([1.0, 4.0], [1.0, 2.0])
    assert t.shape == (2, 2, 3)
    assert t[0, 1, 0] == t[1, 0, 0] == 2.0 and t[0, 1, 1] == t[1, 0, 1] == 1.5
    assert t[0, 0, 0] == 1.0 and t[1, 1, 1] == 2.0 and np.all(t[:, :, 2] == 0.0)
    for eps, sig in (([1.0], [1.0, 2.0]), ([-1.0], [1.0]), ([1.0], [0.0]), ([1.0] * 5, [1.0] * 5), ([], [])):
        with pytest.raises(ValueError):
            api.lorentz_berthelot(eps, sig)
