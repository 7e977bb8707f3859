"""GPU parity of the moment filter (Eq. moment1/moment2) and its transpose
against the oracle, through the C ABI."""
import numpy as np
import pytest
import torch

from oracle import pipeline as P

pytestmark = pytest.mark.gpu


def moment_maps(n, S, seed):
    rng = np.random.default_rng(seed)
    z = rng.uniform(0.2, 0.7, (n, S, S))
    # occluder blobs: a second depth level over part of each map
    mask = rng.random((n, S, S)) < 0.3
    z = np.where(mask, z * 0.6, z)
    return np.stack([z, z * z], 1).astype(np.float32)


def oracle_filter(maps, kind, k, sigma, adjoint):
    w = P.filter_taps(kind, k, sigma)
    out = []
    for m in maps:
        x = torch.as_tensor(m.astype(np.float64))
        if not adjoint:
            out.append(P.filter_separable(x, w).numpy())
        else:
            xr = torch.zeros_like(x, requires_grad=True)
            (g,) = torch.autograd.grad((P.filter_separable(xr, w) * x).sum(), xr)
            out.append(g.numpy())
    return np.stack(out)


@pytest.mark.parametrize('kind,k,sigma,S,n', [
    ('box', 5, 0.0, 200, 2), ('gaussian', 7, 2.0, 131, 3), ('gaussian', 11, 10 / 3, 97, 1),
    ('box', 1, 0.0, 64, 1), ('gaussian', 31, 0.0, 70, 1), ('gaussian', 9, 8 / 3, 256, 1)])
@pytest.mark.parametrize('adjoint', [False, True])
def test_filter_matches_oracle(kind, k, sigma, S, n, adjoint):
    from paper_2308_10896_amd import dsm
    maps = moment_maps(n, S, seed=k * 100 + S)
    got = dsm.filter_moments(torch.as_tensor(maps).cuda(), kind, k, sigma, adjoint).cpu().numpy()
    want = oracle_filter(maps, kind, k, sigma, adjoint)
    np.testing.assert_allclose(got, want, rtol=1e-4, atol=1e-6)


def test_filter_full_size_batch_sampled():
    """64 maps of 512^2 with the 5x5 box filter (batched pose workload):
    every map checked on a sample of rows against the oracle."""
    from paper_2308_10896_amd import dsm
    n, S = 64, 512
    maps = moment_maps(n, S, seed=11)
    got = dsm.filter_moments(torch.as_tensor(maps).cuda(), 'box', 5, 0.0).cpu().numpy()
    w = P.filter_taps('box', 5, 0.0)
    rng = np.random.default_rng(0)
    for i in rng.choice(n, 6, replace=False):
        want = P.filter_separable(torch.as_tensor(maps[i].astype(np.float64)), w).numpy()
        np.testing.assert_allclose(got[i], want, rtol=1e-4, atol=1e-6)


def test_filter_rejects_bad_arguments():
    from paper_2308_10896_amd import dsm, _lib
    x = torch.zeros(1, 2, 16, 16, device='cuda')
    for kw in (dict(k=4), dict(k=33), dict(k=17)):
        with pytest.raises(_lib.DSMError):
            dsm.filter_moments(x, 'box', **kw)
