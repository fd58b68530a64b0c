"""The compact fourth-order pair on the GPU (hs_compact_apply) against the
oracle (or_compact_apply) and against its closed-form eigenvalues at full
size.  Single-operator tolerance: 1e-13 relative in the max norm, as for the
other operators."""
import math

import numpy as np
import pytest

import oracle
from paper_1307_7867_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("n", [1, 3, 7, 15, 31, 63, 127])
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (0.0, 1.0), (1.0, -0.004)])
def test_compact_apply_parity(torch, n, alpha, beta):
    from paper_1307_7867_amd import heatst as hs
    us = [inputs.random_field(n, 20 + b) for b in range(2)]
    u = torch.from_numpy(np.concatenate([x.ravel() for x in us])).cuda()
    y = torch.empty_like(u)
    print(f"compact_apply n={n} alpha={alpha} beta={beta}", flush=True)
    hs.compact_apply(u, y, n, 2, alpha, beta)
    got = y.cpu().numpy()
    for b in range(2):
        ref = oracle.compact_apply(us[b], alpha, beta)
        assert rel(got[b * n ** 3:(b + 1) * n ** 3].reshape(n, n, n), ref) <= 1e-13, (n, b)


def test_compact_apply_eigenvalues_at_255(torch):
    """On a sine mode of a 255^3 grid both matrices act as their closed-form
    eigenvalues (an identity that holds at any size)."""
    from paper_1307_7867_amd import heatst as hs
    n, k = 255, (3, 200, 7)
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) / (n + 1)
    phi = (np.sin(k[2] * np.pi * x)[:, None, None] * np.sin(k[1] * np.pi * x)[None, :, None]
           * np.sin(k[0] * np.pi * x)[None, None, :])
    c = [math.cos(kk * math.pi * h) for kk in k]
    la = (4 * sum(c) + 4 * (c[0] * c[1] + c[0] * c[2] + c[1] * c[2]) - 24) / (6 * h * h)
    lb = 0.5 + sum(c) / 6
    u = torch.from_numpy(phi.ravel()).cuda()
    y = torch.empty_like(u)
    print(f"compact_apply eigen n={n}", flush=True)
    hs.compact_apply(u, y, n, 1, 0.0, 1.0)
    assert np.abs(y.cpu().numpy() - la * phi.ravel()).max() <= 1e-11 * abs(la)
    hs.compact_apply(u, y, n, 1, 1.0, 0.0)
    assert np.abs(y.cpu().numpy() - lb * phi.ravel()).max() <= 1e-13
