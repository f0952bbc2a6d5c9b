"""GPU parity of the BLAS-1 calls (add, axpy, xmul, dot) against the CPU oracle.

add / axpy / xmul are single IEEE roundings, so they must match bit for bit
(NaN-ness compared, payloads not).  dot must be within 1e-13 relative of the
oracle's compensated sum (normalised by sum |x_i y_i| for cancelling data)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2112_10823_amd import cgx

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 7, 4096, 1000003]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def same_bits(a, b):
    a, b = np.asarray(a), np.asarray(b)
    nan = np.isnan(a)
    if not np.array_equal(nan, np.isnan(b)):
        return False
    return np.array_equal(a[~nan].view(np.int64), b[~nan].view(np.int64))


def specials(n, seed):
    v = synth.uniform(seed, n) * np.exp2(np.arange(n) % 61 - 30)
    s = [0.0, -0.0, 5e-324, -5e-324, 2.2250738585072014e-308, 1e-310, np.inf, -np.inf, np.nan,
         1e308, -1e308, 1.0]
    v[: min(n, len(s))] = s[: min(n, len(s))]
    return v


@pytest.mark.parametrize("n", SIZES)
def test_add_xmul_bit_exact(n):
    x, y = synth.uniform(synth.SEED_VEC_X, n), synth.uniform(synth.SEED_VEC_Y, n)
    dx, dy = dev(x), dev(y)
    assert same_bits(cgx.add(dx, dy).cpu().numpy(), oracle.add(x, y))
    assert same_bits(cgx.xmul(dx, dy).cpu().numpy(), oracle.xmul(x, y))


def test_add_xmul_special_values_and_subnormals():
    x, y = specials(1001, 3), specials(1001, 4)[::-1].copy()
    dx, dy = dev(x), dev(y)
    assert same_bits(cgx.add(dx, dy).cpu().numpy(), oracle.add(x, y))
    assert same_bits(cgx.xmul(dx, dy).cpu().numpy(), oracle.xmul(x, y))
    # signed zeros
    z = cgx.add(dev(np.array([-0.0, 0.0, -0.0])), dev(np.array([-0.0, -0.0, 0.0]))).cpu().numpy()
    assert list(np.signbit(z)) == [True, False, False]


@pytest.mark.parametrize("n", SIZES)
def test_axpy_bit_exact_fma(n):
    x, y = synth.uniform(synth.SEED_VEC_X, n), synth.uniform(synth.SEED_VEC_Y, n)
    alpha = -0.7390851332151607
    dy = dev(y)
    cgx.axpy(alpha, dev(x), dy)
    assert same_bits(dy.cpu().numpy(), oracle.axpy(alpha, x, y))


def test_unaligned_and_aliased_operands():
    n = 10001
    x, y = synth.uniform(5, n + 1), synth.uniform(6, n + 1)
    dx, dy = dev(x), dev(y)
    # offset by one element: 8-byte but not 16-byte aligned
    xs, ys = dx[1:], dy[1:]
    assert xs.data_ptr() % 16 == 8
    assert same_bits(cgx.add(xs, ys).cpu().numpy(), oracle.add(x[1:], y[1:]))
    assert same_bits(cgx.xmul(xs, dy[:-1]).cpu().numpy(), oracle.xmul(x[1:], y[:-1]))
    # z aliases x exactly
    z = dx.clone()
    cgx.add(z, dy, z)
    assert same_bits(z.cpu().numpy(), oracle.add(x, y))
    z = dy.clone()
    cgx.xmul(dx, z, z)
    assert same_bits(z.cpu().numpy(), oracle.xmul(x, y))


def test_empty_vectors():
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    assert cgx.add(e, e).numel() == 0
    assert cgx.dot(e, e).item() == 0.0


@pytest.mark.parametrize("n", SIZES + [1 << 22])
def test_dot_relative_1e13(n):
    x, y = synth.uniform(synth.SEED_VEC_X, n), synth.uniform(synth.SEED_VEC_Y, n)
    d = cgx.dot(dev(x), dev(y)).item()
    ref = oracle.dot(x, y)
    scale = max(abs(ref), float(np.sum(np.abs(x * y))) * 1e-3)
    assert abs(d - ref) <= 1e-13 * scale


def test_dot_integer_exact_and_cancelling():
    rng = np.random.default_rng(0)
    x = rng.integers(-1000, 1000, 300001).astype(float)
    y = rng.integers(-1000, 1000, 300001).astype(float)
    assert cgx.dot(dev(x), dev(y)).item() == float(np.dot(x.astype(np.int64), y.astype(np.int64)))
    # strongly cancelling: the compensated GPU sum matches the compensated oracle
    x = synth.uniform(9, 200000)
    y = np.concatenate([x[:100000], -x[:100000]]) * 1e6
    x = np.concatenate([x[:100000], x[:100000]])
    y[7] += 1e-3
    d = cgx.dot(dev(x), dev(y)).item()
    assert abs(d - oracle.dot(x, y)) <= 1e-13 * float(np.sum(np.abs(x * y)))


def test_dot_deterministic():
    x, y = synth.uniform(1, 3000017), synth.uniform(2, 3000017)
    dx, dy = dev(x), dev(y)
    vals = {cgx.dot(dx, dy).item() for _ in range(5)}
    assert len(vals) == 1


def test_blas1_full_size_2pow26():
    """The largest BLAS-1 size of the FP64 microbenchmark (2^26, uniform[-1,1])."""
    n = 1 << 26
    x, y = synth.uniform(synth.SEED_VEC_X, n), synth.uniform(synth.SEED_VEC_Y, n)
    dx, dy = dev(x), dev(y)
    assert same_bits(cgx.add(dx, dy).cpu().numpy(), oracle.add(x, y))
    assert same_bits(cgx.xmul(dx, dy).cpu().numpy(), oracle.xmul(x, y))
    d = cgx.dot(dx, dy).item()
    ref = oracle.dot(x, y)
    assert abs(d - ref) <= 1e-13 * abs(ref)
    cgx.axpy(0.5, dx, dy)
    assert same_bits(dy.cpu().numpy(), oracle.axpy(0.5, x, y))


def test_demote_round_to_nearest():
    x = specials(20001, 8)
    assert same_bits(cgx.demote(dev(x)).cpu().numpy().astype(np.float64),
                     x.astype(np.float32).astype(np.float64))


@pytest.mark.parametrize("n", [0, 1, 4096, 1000003])
def test_dot_sync_equals_dot(n):
    """cgx_dot_sync returns to the host exactly the bits cgx_dot writes to the
    device, and is within the dot bar of the oracle's compensated sum."""
    x = synth.uniform(31, n)
    y = synth.uniform(32, n)
    dx, dy = dev(x), dev(y)
    ds = cgx.dot_sync(dx, dy)
    dd = cgx.dot(dx, dy).item()
    assert np.float64(ds).view(np.int64) == np.float64(dd).view(np.int64)
    if n:
        ref = oracle.dot(x, y)
        assert abs(ds - ref) <= 1e-13 * max(abs(ref), 1e-3 * float(np.sum(np.abs(x * y))))
    else:
        assert ds == 0.0


def test_dot_sync_integer_exact():
    rng = np.random.default_rng(5)
    x = rng.integers(-1000, 1000, 100000).astype(np.float64)
    y = rng.integers(-1000, 1000, 100000).astype(np.float64)
    assert cgx.dot_sync(dev(x), dev(y)) == float(np.dot(x.astype(np.int64), y.astype(np.int64)))
