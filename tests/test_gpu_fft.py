"""Parity of the Fourier-magnitude feature kernel (hloc_fft_features_async)
with the FP64 oracle, which writes the discrete Fourier transform out from its
definition, on seeded panoramic signals and special rows.

Bound used (u = 2^-53): the kernel's FP64 radix-2 transform of the packed
signal errs by at most about 8 u log2(n) sqrt(n) ||x||_2 per bin (twiddles
within 2u), the unpacking doubles that and adds a few u sqrt(n) ||x||_2; the
oracle's direct sums err by at most about (L + 16) u ||x||_1. With E the sum
of both, the kernel's result, rounded once to fp32, lies within
2^-24 |oracle| + 1.01 E of the oracle, and E is far below an fp32 ulp of
every bin these signals produce, so almost every value is the oracle's
rounded to fp32 exactly."""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2006_08861_amd import hloc, workload

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(hloc.LIB_PATH):
        pytest.fail("libhloc.so is not built")
    return torch


def tolerance(x: np.ndarray, ora: np.ndarray) -> np.ndarray:
    L = x.shape[1]
    n = L // 2
    l2 = np.sqrt((x.astype(np.float64) ** 2).sum(axis=1, keepdims=True))
    l1 = np.abs(x.astype(np.float64)).sum(axis=1, keepdims=True)
    e = 16.0 * (math.log2(n) + 2.0) * math.sqrt(n) * U * l2 + (L + 16.0) * U * l1
    return 2.0 ** -24 * np.abs(ora) + 1.01 * e + 2.0 ** -149


def check(x: np.ndarray, d: int, got: np.ndarray, name: str, min_exact: float = 0.999):
    ora = oracle.fft_magnitude(x, d)
    assert got.shape == ora.shape and got.dtype == np.float32, name
    err = np.abs(got.astype(np.float64) - ora)
    tol = tolerance(x, ora)
    bad = np.argwhere(err > tol)
    assert bad.size == 0, (f"{name}: {len(bad)} values beyond the bound, first {bad[0]}: "
                           f"{got[tuple(bad[0])]} vs {ora[tuple(bad[0])]}")
    exact = float(np.mean(got == ora.astype(np.float32)))
    assert exact >= min_exact, f"{name}: only {exact:.4f} equal to the rounded oracle"


def _signals(n, length, seed):
    return workload.panoramic_signals(n, length, np.random.default_rng(seed))


@pytest.mark.parametrize("length,d,nsig", [(2, 2, 5), (4, 3, 7), (8, 1, 64), (64, 33, 1000),
                                           (128, 65, 333), (128, 20, 9), (256, 129, 100),
                                           (512, 256, 4099), (512, 257, 300), (512, 100, 3),
                                           (1024, 100, 777), (2048, 1025, 257)])
def test_fft_parity(torch_cuda, length, d, nsig):
    x = _signals(nsig, length, 1000 + length + d)
    got = hloc.fft_features(torch_cuda.from_numpy(x).cuda(), d).cpu().numpy()
    check(x, d, got, f"len={length} d={d} nsig={nsig}")


def test_fft_special_rows(torch_cuda):
    """Zeros, constants, pure tones, alternating signs, tiny and huge scales in
    one batch."""
    L, d = 256, 129
    t = np.arange(L)
    rows = [np.zeros(L), np.full(L, 3.0), np.full(L, -1e-30), np.cos(2 * np.pi * 5 * t / L),
            7.5 * np.sin(2 * np.pi * 127 * t / L + 0.3), (-1.0) ** t, np.where(t == 17, 1.0, 0.0),
            1e30 * np.random.default_rng(3).standard_normal(L),
            1e-30 * np.random.default_rng(4).standard_normal(L)]
    x = np.stack(rows).astype(np.float32)
    got = hloc.fft_features(x, d)
    check(x, d, got, "special rows", min_exact=0.3)
    assert got[0].max() == 0.0
    assert got[6].tolist() == [1.0] * d  # a unit impulse has a flat spectrum of 1


def test_fft_rotation_invariance(torch_cuda):
    """A rotated panorama (circular shift) gives the same feature within the
    bound of each against the oracle."""
    x = _signals(64, 512, 5)
    f = hloc.fft_features(x, 256)
    for s in (1, 100, 511):
        g = hloc.fft_features(np.ascontiguousarray(np.roll(x, s, axis=1)), 256)
        ora = oracle.fft_magnitude(x, 256)
        assert np.all(np.abs(g.astype(np.float64) - f) <= 2 * tolerance(x, ora)), s


def test_fft_empty_and_stream(torch_cuda):
    torch = torch_cuda
    assert hloc.fft_features(torch.empty((0, 8), device="cuda"), 4).shape == (0, 4)
    x = _signals(300, 128, 9)
    s = torch.cuda.Stream()
    xd = torch.from_numpy(x).cuda()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        got = hloc.fft_features(xd, 65, stream=s)
    s.synchronize()
    check(x, 65, got.cpu().numpy(), "side stream")


def test_fft_full_size_sampled(torch_cuda):
    """200,000 signals of 512 samples to 256 bins (the database of the
    fp32-200k-d256 workload, the launch the benchmark times): every value
    finite, 2,000 seeded rows against the oracle."""
    torch = torch_cuda
    x = _signals(200_000, 512, 77)
    got = hloc.fft_features(torch.from_numpy(x).cuda(), 256).cpu().numpy()
    assert np.isfinite(got).all()
    rows = np.sort(np.random.default_rng(78).choice(len(x), 2000, replace=False))
    rows = np.concatenate([[0, len(x) - 1], rows])
    check(x[rows], 256, got[rows], "200k x 512 sampled")
