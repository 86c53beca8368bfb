"""CPU model of the pruned 3-D transforms (no GPU).

Re-derives, in numpy with the kernels' own index arithmetic, that
  * the in-place radix-2 decimation-in-time pass (bit-reversed input) gives
    the forward DFT in natural order, and the decimation-in-frequency pass
    (natural input) gives the inverse DFT in bit-reversed order;
  * the pruned chain  x r2c (modes 0..K) -> y (keep |my| <= K) -> z + spectral
    operator + inverse z -> zero-padded inverse y -> Hermitian c2r along x
    equals full transforms with every mode outside |m_i| <= K zeroed.
"""
import numpy as np
import pytest


def bitrev(j, logn):
    return int(format(j, f"0{logn}b")[::-1], 2)


def tw(n, sign):
    k = np.arange(n // 2)
    return np.exp(sign * 2j * np.pi * k / n)


def fft_dit(buf, logn, t):
    """buf[j, s]: element j of sequence s (bit-reversed order on entry)."""
    n = 1 << logn
    for s in range(1, logn + 1):
        lh = s - 1
        half = 1 << lh
        tsh = logn - s
        for k in range(n // 2):
            j = k & (half - 1)
            i0 = ((k >> lh) << (lh + 1)) + j
            i1 = i0 + half
            w = t[j << tsh]
            a, v = buf[i0].copy(), buf[i1].copy()
            buf[i0] = a + w * v
            buf[i1] = a - w * v


def fft_dif(buf, logn, t):
    n = 1 << logn
    for s in range(logn, 0, -1):
        lh = s - 1
        half = 1 << lh
        tsh = logn - s
        for k in range(n // 2):
            j = k & (half - 1)
            i0 = ((k >> lh) << (lh + 1)) + j
            i1 = i0 + half
            w = t[j << tsh]
            a, v = buf[i0].copy(), buf[i1].copy()
            buf[i0] = a + v
            buf[i1] = (a - v) * w


@pytest.mark.parametrize("logn", [1, 3, 4, 6])
def test_dit_and_dif_passes(logn):
    n = 1 << logn
    rng = np.random.default_rng(logn)
    x = rng.normal(size=(n, 3)) + 1j * rng.normal(size=(n, 3))
    b = np.empty_like(x)
    for j in range(n):
        b[bitrev(j, logn)] = x[j]
    fft_dit(b, logn, tw(n, -1))
    np.testing.assert_allclose(b, np.fft.fft(x, axis=0), rtol=1e-12, atol=1e-12)
    b = x.copy()
    fft_dif(b, logn, tw(n, +1))
    out = np.empty_like(b)
    for j in range(n):
        out[j] = b[bitrev(j, logn)]
    np.testing.assert_allclose(out, np.fft.ifft(x, axis=0) * n, rtol=1e-12, atol=1e-12)


def spectral(G, mx, my, mz, K, op):
    """The operator on one mode (any function of the 3 components); zero
    outside |m_i| <= K and at k = 0."""
    if abs(mz) > K or abs(my) > K or mx > K or (mx == 0 and my == 0 and mz == 0):
        return np.zeros(3, complex)
    return op(G, mx, my, mz)


def op_curl(G, mx, my, mz):
    k = np.array([mx, my, mz], float)
    f = np.exp(-k @ k / 50.0) / (k @ k) * (1 + 0.1 * mx + 0.01 * abs(my) + 0.001 * abs(mz))
    return 1j * np.cross(k, G) * f


@pytest.mark.parametrize("n,K", [(8, 2), (16, 4), (16, 5)])
def test_pruned_chain_equals_masked_full_transforms(n, K):
    rng = np.random.default_rng(n + K)
    logn = int(np.log2(n))
    g = rng.normal(size=(3, n, n, n))             # [c][z][y][x]
    K1, NY = K + 1, 2 * K + 1
    twf, twi = tw(n, -1), tw(n, +1)
    # x forward: rows (c, z, y), modes 0..K -> A[c][z][y][kx]
    A = np.empty((3, n, n, K1), complex)
    for c in range(3):
        for z in range(n):
            for y in range(n):
                b = np.empty(n, complex)
                for j in range(n):
                    b[bitrev(j, logn)] = g[c, z, y, j]
                fft_dit(b, logn, twf)
                A[c, z, y] = b[:K1]
    # y forward -> B[c][my+K][z][kx]
    B = np.empty((3, NY, n, K1), complex)
    for c in range(3):
        for z in range(n):
            b = np.empty((n, K1), complex)
            for y in range(n):
                b[bitrev(y, logn)] = A[c, z, y]
            fft_dit(b, logn, twf)
            for myp in range(NY):
                B[c, myp, z] = b[(myp - K) % n]
    # z forward, operator, z inverse (bit-reversed), per (my, kx)
    for myp in range(NY):
        b = np.empty((n, 3, K1), complex)
        for z in range(n):
            b[bitrev(z, logn)] = B[:, myp, z, :]
        fft_dit(b, logn, twf)
        for z in range(n):
            mz = z if z <= n // 2 else z - n
            for q in range(K1):
                b[z, :, q] = spectral(b[z, :, q], q, myp - K, mz, K, op_curl)
        fft_dif(b, logn, twi)
        for z in range(n):
            B[:, myp, z, :] = b[bitrev(z, logn)]
    # y inverse (zero padded) -> A[c][z][y][kx]
    for c in range(3):
        for z in range(n):
            b = np.zeros((n, K1), complex)
            for y in range(n):
                my = y if y <= n // 2 else y - n
                if -K <= my <= K:
                    b[y] = B[c, my + K, z]
            fft_dif(b, logn, twi)
            for y in range(n):
                A[c, z, y] = b[bitrev(y, logn)]
    # x inverse: Hermitian completion, real part
    out = np.empty_like(g)
    for c in range(3):
        for z in range(n):
            for y in range(n):
                b = np.zeros(n, complex)
                for m in range(n):
                    if m < K1:
                        b[m] = A[c, z, y, m]
                    elif n - m < K1:
                        b[m] = np.conj(A[c, z, y, n - m])
                fft_dif(b, logn, twi)
                out[c, z, y] = [b[bitrev(j, logn)].real for j in range(n)]
    # reference: full r2c, the operator on the half space, full c2r
    G = np.fft.rfftn(g, axes=(1, 2, 3))           # [c][z][y][x half]
    V = np.zeros_like(G)
    for iz in range(n):
        mz = iz if iz <= n // 2 else iz - n
        for iy in range(n):
            my = iy if iy <= n // 2 else iy - n
            for ix in range(n // 2 + 1):
                V[:, iz, iy, ix] = spectral(G[:, iz, iy, ix], ix, my, mz, K, op_curl)
    ref = np.fft.irfftn(V, s=(n, n, n), axes=(1, 2, 3)) * n ** 3
    np.testing.assert_allclose(out, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())
