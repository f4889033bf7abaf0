"""Host-side checks of the autograd binding (no GPU needed)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def test_log_marginal_refuses_the_information_sharing_start():
    # the information-sharing start scales I0 for PEs other than the first;
    # the reverse sweep differentiates a shift, so the binding refuses it
    from paper_1310_4624_amd import PF_INIT_INFOSHARE
    from paper_1310_4624_amd.grad import log_marginal
    theta = torch.tensor([1.5, 10.0, 0.5], dtype=torch.float64)
    with pytest.raises(ValueError):
        log_marginal(theta, torch.zeros((2, 8, 8)), dict(init_mode=PF_INIT_INFOSHARE),
                     np.zeros((1, 5), np.float32))
