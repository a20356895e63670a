"""The study module's own input generator (the paper's Sec. 5.1 recipe)
draws exactly the arrays of the shared test generator, so the study's
figures refer to the inputs the parity tests use."""

import numpy as np
import pytest

import workloads as wl


@pytest.mark.parametrize("phi", [0.0, 1.0, 4.0])
@pytest.mark.parametrize("n,batch,seed", [(16, 1, 0), (1000, 3, 5)])
def test_study_inputs_equal_shared_generator(phi, n, batch, seed):
    from paper_2603_29129_amd import study
    a = study.inputs(n, phi, seed=seed, batch=batch)
    b = wl.paper_phi(n, phi, seed=seed, batch=batch)
    assert a.dtype == b.dtype and a.shape == b.shape
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
