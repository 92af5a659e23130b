"""Per-class sums, naive Bayes and GDA training (paper section 4.2
applications on the section 2.3 per-label reduce) against the FP64 oracle
(needs an MI355X).

Bars, derived from the arithmetic:
  - counts and priors: exact (integers, one division each);
  - sums of integer-valued features (naive Bayes counts): exact, so phi,
    computed from them with the oracle's operations in the oracle's order,
    must be bit-equal;
  - sums of real features: the GPU and the oracle add the same terms in
    different orders, each within (m - 1) u sum|x| of the exact sum
    (m terms, u = 2^-53), so they differ by at most 2 (m - 1) u sum|x|;
  - GDA covariance: each element is (1/n) sum_i z_ia z_ib; two summation
    orders differ by at most 2 n u (1/n) sum_i |z_ia z_ib| <=
    2 n u sqrt(S_aa S_bb) (Cauchy-Schwarz), plus the effect of the means'
    last-bit differences, covered by a factor of 2 and 1e-14 of the
    largest element.
"""
import sys

import numpy as np
import pytest

from oracle import ml
from paper_1109_0778_amd import datagen

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _plan(B, n, d, k):
    return B.Plan(n, d, k)


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("n,d,k", [(1, 1, 1), (7, 3, 2), (1000, 16, 5), (4099, 64, 64), (20000, 37, 300),
                                   (3000, 128, 1024), (5000, 200, 7)])
def test_class_sums(n, d, k):
    torch = _torch()
    from paper_1109_0778_amd import binding as B
    say(f"class sums n={n} d={d} k={k}")
    X, y = datagen.gda_classes(n, d, min(k, max(1, n)), seed=n + d)
    y = (y % k).astype(np.int32)
    plan = _plan(B, n, d, k)
    S = torch.empty((k, d), dtype=torch.float64, device="cuda")
    cnt = torch.empty(k, dtype=torch.int64, device="cuda")
    B.km_class_sums(plan, _dev(torch, X), _dev(torch, y), S, cnt)
    torch.cuda.synchronize()
    S_o, c_o = ml.class_sums(X, y, k)
    assert np.array_equal(cnt.cpu().numpy(), c_o)
    absum = np.zeros((k, d))
    np.add.at(absum, y, np.abs(X.astype(np.float64)))
    lim = 2.0 * np.maximum(c_o[:, None] - 1, 0) * U * absum
    err = np.abs(S.cpu().numpy() - S_o)
    assert np.all(err <= lim), f"max excess {(err - lim).max():.3e}"
    # integer features: exact
    Xi, yi = datagen.nb_counts(n, d, k, seed=3)
    B.km_class_sums(plan, _dev(torch, Xi), _dev(torch, yi), S, cnt)
    torch.cuda.synchronize()
    S_o, c_o = ml.class_sums(Xi, yi, k)
    assert np.array_equal(S.cpu().numpy(), S_o)
    assert np.array_equal(cnt.cpu().numpy(), c_o)


@pytest.mark.parametrize("n,d,k", [(1, 1, 1), (50, 4, 9), (10000, 64, 20), (4097, 100, 3), (30000, 16, 200),
                                   (1 << 20, 64, 16)])
def test_naive_bayes_bit_exact(n, d, k):
    torch = _torch()
    from paper_1109_0778_amd import binding as B
    say(f"naive Bayes n={n} d={d} k={k}")
    X, y = datagen.nb_counts(n, d, k, seed=d + k)
    plan = _plan(B, n, d, k)
    prior = torch.empty(k, dtype=torch.float64, device="cuda")
    phi = torch.empty((k, d), dtype=torch.float64, device="cuda")
    B.nb_train(plan, _dev(torch, X), _dev(torch, y), prior, phi)
    torch.cuda.synchronize()
    p_o, phi_o = ml.nb_train(X, y, k)
    assert np.array_equal(prior.cpu().numpy(), p_o)
    assert np.array_equal(phi.cpu().numpy(), phi_o)
    assert np.allclose(phi.cpu().numpy().sum(1), 1.0, rtol=1e-12)


def test_naive_bayes_validate_rejects_bad_labels():
    torch = _torch()
    from paper_1109_0778_amd import binding as B
    X, y = datagen.nb_counts(1000, 8, 4, seed=1)
    y[17] = 4
    plan = _plan(B, 1000, 8, 4)
    plan.set_validate(True)
    prior = torch.full((4,), -1.0, dtype=torch.float64, device="cuda")
    phi = torch.full((4, 8), -1.0, dtype=torch.float64, device="cuda")
    with pytest.raises(B.KMeansError):
        B.nb_train(plan, _dev(torch, X), _dev(torch, y), prior, phi)
    torch.cuda.synchronize()
    assert (prior.cpu().numpy() == -1.0).all() and (phi.cpu().numpy() == -1.0).all()


def _gda_check(torch, B, n, d, k, seed):
    X, y = datagen.gda_classes(n, d, k, seed)
    plan = _plan(B, n, d, k)
    prior = torch.empty(k, dtype=torch.float64, device="cuda")
    mu = torch.empty((k, d), dtype=torch.float64, device="cuda")
    sigma = torch.empty((d, d), dtype=torch.float64, device="cuda")
    B.gda_train(plan, _dev(torch, X), _dev(torch, y), prior, mu, sigma)
    torch.cuda.synchronize()
    p_o, mu_o, s_o = ml.gda_train(X, y, k)
    assert np.array_equal(prior.cpu().numpy(), p_o)
    cnt = np.bincount(y, minlength=k)
    absum = np.zeros((k, d))
    np.add.at(absum, y, np.abs(X.astype(np.float64)))
    mlim = 2.0 * np.maximum(cnt[:, None] - 1, 0) * U * absum / np.maximum(cnt[:, None], 1) + 2 * U * np.abs(mu_o)
    assert np.all(np.abs(mu.cpu().numpy() - mu_o) <= mlim)
    S = sigma.cpu().numpy()
    dg = np.sqrt(np.abs(np.diag(s_o)))
    lim = 4.0 * n * U * np.outer(dg, dg) + 1e-14 * np.abs(s_o).max()
    err = np.abs(S - s_o)
    assert np.all(err <= lim), f"sigma error {err.max():.3e}, worst excess {(err - lim).max():.3e}"
    assert np.array_equal(S, S.T), "sigma must be symmetric"
    return err.max() / max(np.abs(s_o).max(), 1e-300)


@pytest.mark.parametrize("n,d,k", [(1, 1, 1), (9, 5, 3), (1000, 16, 4), (5000, 64, 10), (4099, 65, 2),
                                   (3000, 100, 7), (2000, 128, 12), (1500, 200, 5)])
def test_gda(n, d, k):
    torch = _torch()
    from paper_1109_0778_amd import binding as B
    say(f"GDA n={n} d={d} k={k}")
    rel = _gda_check(torch, B, n, d, k, seed=n * 7 + d)
    say(f"  sigma max error / max |sigma| = {rel:.2e}")


@pytest.mark.slow
def test_gda_full_size():
    """n = 2^20 samples, d = 64, k = 16 classes."""
    torch = _torch()
    from paper_1109_0778_amd import binding as B
    rel = _gda_check(torch, B, 1 << 20, 64, 16, seed=5)
    say(f"GDA n=2^20: sigma max error / max |sigma| = {rel:.2e}")
