"""The identity that lets split-length transforms derive the Hankel chirp spectrum from the
Toeplitz one (Sec. 3.1, the DST and DCT through chirp-z convolutions).

With the chirp c_d = exp(i pi d^2 / D) and M = D/2, c_{M+e} = e^{i pi M/2} (-1)^e c_e, so the
Hankel window (c_{d+2} on d in [0, 2N-2] for the sine transform, -c_d for the cosine
transform) is the Toeplitz window (c_d on d in [1-N, N-1]) moved by s = N - 1 positions and
modulated by (-1)^e: K2_q = phi w^{s q} K1_{q+P/2}, w = exp(-2 pi i/P).  The device builds
the phase as a table entry for q mod 64 times one for q div 64 (element 0 of a thread) and
per-element steps w^{s D i}; these tests check both the identity and that factorisation in
FP64, for windows written out from their definitions."""
import numpy as np
import pytest


def _windows(N, bc):
    M = N + 1 if bc == "sine" else N - 1
    D = 2 * M
    P = 128
    while P < 2 * N - 1:
        P *= 2
    d = np.arange(0, 2 * N + 1)
    ch = np.exp(1j * np.pi * ((d * d) % (2 * D)) / D)   # c_d, exact reduction of d^2 mod 2D
    k1 = np.zeros(P, complex)
    k2 = np.zeros(P, complex)
    for e in range(1 - N, N):
        k1[e % P] = ch[abs(e)]
    for e in range(0, 2 * N - 1):
        k2[e % P] = ch[e + 2] if bc == "sine" else -ch[e]
    return M, P, np.fft.fft(k1), np.fft.fft(k2)


def _phi(M, bc):
    return (-1 if bc == "cosine" else 1) * [1, 1j, -1, -1j][M % 4]


@pytest.mark.parametrize("bc", ["sine", "cosine"])
@pytest.mark.parametrize("N", [3, 64, 1000, 4097, 8200, 16000])
def test_hankel_spectrum_is_the_shifted_modulated_toeplitz_spectrum(N, bc):
    M, P, K1, K2 = _windows(N, bc)
    q = np.arange(P)
    pred = _phi(M, bc) * np.exp(-2j * np.pi * (((N - 1) * q) % P) / P) * K1[(q + P // 2) % P]
    assert np.abs(pred - K2).max() <= 1e-11 * np.abs(K2).max()


def test_a_dropped_modulation_breaks_the_identity():
    # the (-1)^e modulation is what moves K1 by half the length: without it the prediction fails
    M, P, K1, K2 = _windows(1000, "sine")
    q = np.arange(P)
    pred = _phi(M, "sine") * np.exp(-2j * np.pi * ((999 * q) % P) / P) * K1
    assert np.abs(pred - K2).max() > 0.1 * np.abs(K2).max()


@pytest.mark.parametrize("N,T", [(9000, 1024), (9000, 512), (16384, 1024), (12000, 512)])
def test_phase_table_factorisation_covers_every_split_position(N, T):
    # split half of P: element i of thread t holds frequency q = 2 (t + i T) + odd; the phase
    # is lo[q0 mod 64] hi[q0 div 64] (q0 = 2t + odd) times the step w^{s 2T i} for i < RT/2,
    # and (-1)^s times that for element i + RT/2 (frequency q + P/2)
    M, P, _, _ = _windows(N, "sine")
    s = N - 1
    w = lambda j: np.exp(-2j * np.pi * (j % P) / P)
    phi = _phi(M, "sine")
    lo = np.array([phi * w(s * k) for k in range(64)])
    hi = np.array([w(64 * s * m) for m in range(P // 64)])
    PE = P // 2
    RT = PE // T
    got = np.zeros(P, complex)
    for odd in (0, 1):
        t = np.arange(T)
        q0 = 2 * t + odd
        base = lo[q0 & 63] * hi[q0 >> 6]
        for i in range(RT // 2):
            step = w(s * 2 * T * i)
            q = 2 * (t + i * T) + odd
            got[q] = base * step
            got[q + PE] = (-1) ** s * base * step
    want = phi * np.exp(-2j * np.pi * ((s * np.arange(P)) % P) / P)
    assert np.abs(got - want).max() < 1e-12
