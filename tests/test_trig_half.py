"""The length-N forms of the DCT-I and DST-I that the FP64 PPE kernels use
reproduce the DFT of the even / odd extension of length 2N (numpy FFT as the
reference), for odd and even N, with the running sums taken in chunks and a
start value as the kernels take them."""
import numpy as np
import pytest


def half_length(f, sine, chunk):
    N = len(f) - 1
    j = np.arange(N)
    s = np.sin(np.pi * j / N)
    fr = f[N - j]
    if sine:
        y = s * (f[:N] + fr) + 0.5 * (f[:N] - fr)
    else:
        y = 0.5 * (f[:N] + fr) - s * (f[:N] - fr)
    Y = np.fft.fft(y)
    Yr = Y[(-np.arange(N)) % N]
    H = N // 2
    k = np.arange(H + 1)
    out = np.zeros(N + 1, complex)
    if sine:
        out[2 * k] = np.where(k == 0, 0, Y[k] - Yr[k])
        terms = np.where(k == 0, Y[0], Y[k] + Yr[k])
        start = 0.0
    else:
        out[2 * k] = Y[k] + Yr[k]
        terms = np.where(k == 0, 0, 1j * (Y[k] - Yr[k]))
        start = f[0] - f[N] + 2 * np.sum(f[1:N] * np.cos(np.pi * np.arange(1, N) / N))
    # running sum in chunks: chunk-local sums, then the sums of earlier chunks
    run = np.zeros(H + 1, complex)
    carry = start
    for c0 in range(0, H + 1, chunk):
        part = np.cumsum(terms[c0:c0 + chunk])
        run[c0:c0 + chunk] = part + carry
        carry = carry + part[-1]
    odd = 2 * k + 1 <= N
    out[2 * k[odd] + 1] = -1j * run[odd] if sine else run[odd]
    return out


@pytest.mark.parametrize("sine", [False, True])
@pytest.mark.parametrize("N", [2, 3, 4, 5, 8, 63, 64, 95, 1023, 1024])
def test_length_n_trig_transforms(sine, N):
    rng = np.random.default_rng(N + 7 * sine)
    f = rng.standard_normal(N + 1) + 1j * rng.standard_normal(N + 1)
    if sine:
        f[0] = f[N] = 0.0
    ext = np.concatenate([f, (-1.0 if sine else 1.0) * f[N - 1:0:-1]])
    Z = np.fft.fft(ext)[:N + 1]
    for chunk in (1, 3, 64):
        got = half_length(f, sine, chunk)
        assert np.abs(got - Z).max() <= 1e-13 * np.abs(Z).max(), (sine, N, chunk)
