"""The fp64 network oracle pinned by finite differences (CPU)."""
import numpy as np

from oracle import mlp as OM


def test_param_count_matches_header():
    import re, os
    h = open(os.path.join(os.path.dirname(__file__), "..", "include", "crfrob.h")).read()
    assert int(re.search(r"#define CR_MLP_PARAMS (\d+)", h).group(1)) == OM.NPARAM


def test_gradient_by_central_differences():
    rng = np.random.default_rng(7)
    w = OM.init(3)
    x = rng.uniform(-1, 2, (9, OM.IN))
    t = rng.uniform(0, 1, 9)
    g, L = OM.grad(w, x, t)
    assert abs(L - OM.loss(w, x, t)) < 1e-12
    # one coordinate in every parameter block, plus random ones
    blocks = [0, OM.IN * OM.HID + 5, OM.IN * OM.HID + OM.HID + 777, OM.NPARAM - OM.HID - 2 - 3,
              OM.NPARAM - 3, OM.NPARAM - 1]
    idx = blocks + list(rng.integers(0, OM.NPARAM, 20))
    h = 1e-6
    for i in idx:
        e = np.zeros(OM.NPARAM)
        e[i] = h
        fd = (OM.loss(w + e, x, t) - OM.loss(w - e, x, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * (1 + abs(g[i])), (i, fd, g[i])


def test_forward_special_cases():
    # all-zero weights: the output is b3; identity-like one-unit path
    w = np.zeros(OM.NPARAM)
    w[-1] = 0.25
    assert np.allclose(OM.forward(w, np.ones((3, OM.IN))), 0.25)
    W1, b1, W2, b2, w3, b3 = OM.unpack(w)
    w2 = w.copy()
    w2[0 * OM.HID + 0] = 2.0                            # W1[0][0]
    w2[OM.IN * OM.HID + OM.HID + 0 * OM.HID + 0] = 3.0  # W2[0][0]
    w2[OM.NPARAM - OM.HID - 1 + 0] = 0.5                # w3[0]
    x = np.zeros((2, OM.IN))
    x[0, 0] = 1.0
    x[1, 0] = -1.0                                      # killed by the first ReLU
    assert np.allclose(OM.forward(w2, x), [0.25 + 0.5 * 3.0 * 2.0, 0.25])
