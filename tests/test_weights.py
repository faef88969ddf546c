"""The committed guess-network parameters: a plain float32 array of the
parameter layout (read without unpickling), finite, with a non-zero last
layer (a trained correction, not the linear-extrapolation start)."""
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_committed_weights_have_the_parameter_layout():
    from paper_2204_03575_amd.chm import NET_NPARAMS, unflatten_params
    a = np.load(os.path.join(ROOT, "paper_2204_03575_amd", "weights", "guess256.npy"),
                allow_pickle=False)
    assert a.dtype == np.float32 and a.shape == (NET_NPARAMS,)
    assert np.all(np.isfinite(a))
    layers = unflatten_params(a)
    assert [w.shape for w, _ in layers] == [(3, 3, 8, 32), (3, 3, 32, 32), (3, 3, 32, 32), (3, 3, 32, 4)]
    assert np.abs(layers[-1][0]).max() > 0
