"""CPU model of the pruned 3-D transforms (no GPU).

Re-derives, in numpy with the kernels' own index arithmetic, that
  * the Stockham passes (radix 16, 8, 4, 2 in registers, twiddles from a
    full-circle table, balanced radices) give the forward and inverse DFT in
    natural order;
  * the pruned chain  x r2c (modes 0..K) -> y (keep |my| <= K) -> z + spectral
    operator + inverse z -> zero-padded inverse y -> Hermitian c2r along x
    equals full transforms with every mode outside |m_i| <= K zeroed, with
    the forward x transform taking two real rows per complex sequence as the
    kernel does (spectra separated through Z(n - k)).
"""
import numpy as np
import pytest


def tw(n, sign):
    """Full-circle table: tw[k] = exp(sign 2 pi i k / n), k < n."""
    return np.exp(sign * 2j * np.pi * np.arange(n) / n)


def dft_regs(v, sign):
    """Size-R DFT the way the kernel does it: bit-reversed radix-2 decimation
    in time with twiddles exp(sign 2 pi i m / 16)."""
    R = len(v)
    LR = R.bit_length() - 1
    v = [v[int(format(i, f"0{LR}b")[::-1], 2)] for i in range(R)]
    half = 1
    while half < R:
        for k in range(0, R, 2 * half):
            for j in range(half):
                m = j * (8 // half)
                w = np.exp(sign * 2j * np.pi * m / 16)
                a, t = v[k + j], w * v[k + j + half]
                v[k + j], v[k + j + half] = a + t, a - t
        half *= 2
    return v


def stockham_pass(src, dst, n, R, Ns, t, sign):
    """One radix-R pass; src/dst[j] is element j (a row over the batch)."""
    nj = n // R
    step = n // (Ns * R)
    for j in range(nj):
        v = [src[j + r * nj].copy() for r in range(R)]
        jm = j % Ns
        for r in range(1, R):
            v[r] = v[r] * t[jm * r * step]
        v = dft_regs(v, sign)
        d0 = (j - jm) * R + jm
        for r in range(R):
            dst[d0 + r * Ns] = v[r]


def fft_batch(buf, logn, t, sign):
    """Passes of radix <= 16 chosen as the kernel does; returns the result."""
    n = 1 << logn
    a, b = buf.copy(), np.empty_like(buf)
    Ns, rem = 1, logn
    while rem > 0:
        passes = (rem + 3) // 4
        lr = (rem + passes - 1) // passes
        stockham_pass(a, b, n, 1 << lr, Ns, t, sign)
        a, b = b, a
        Ns <<= lr
        rem -= lr
    return a


@pytest.mark.parametrize("logn", [1, 2, 3, 4, 5, 6, 7, 9])
def test_stockham_batches(logn):
    n = 1 << logn
    rng = np.random.default_rng(logn)
    x = rng.normal(size=(n, 3)) + 1j * rng.normal(size=(n, 3))
    np.testing.assert_allclose(fft_batch(x, logn, tw(n, -1), -1), np.fft.fft(x, axis=0),
                               rtol=1e-11, atol=1e-11 * n)
    np.testing.assert_allclose(fft_batch(x, logn, tw(n, +1), +1), np.fft.ifft(x, axis=0) * n,
                               rtol=1e-11, atol=1e-11 * n)


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
    # x forward: rows (c, z, y) two at a time (y even and y + 1 as the real
    # and imaginary parts of one complex sequence), spectra separated with
    # Z(n - k); modes 0..K -> A[c][z][y][kx]
    A = np.empty((3, n, n, K1), complex)
    k = np.arange(K1)
    for c in range(3):
        for z in range(n):
            rows = (g[c, z, 0::2] + 1j * g[c, z, 1::2]).T     # [x][pair]
            Z = fft_batch(rows, logn, twf, -1)                 # [k][pair]
            Zm = np.conj(Z[(n - k) % n])
            A[c, z, 0::2] = ((Z[:K1] + Zm) / 2).T
            A[c, z, 1::2] = ((Z[:K1] - Zm) / 2j).T
    # y forward -> B[c][my+K][z][kx]
    B = np.empty((3, NY, n, K1), complex)
    for c in range(3):
        for z in range(n):
            res = fft_batch(A[c, z], logn, twf, -1)      # [y][kx]
            for myp in range(NY):
                B[c, myp, z] = res[(myp - K) % n]
    # z forward, operator, z inverse, per (my, kx)
    for myp in range(NY):
        buf = np.moveaxis(B[:, myp], 1, 0).copy()       # [z][c][kx]
        res = fft_batch(buf, logn, twf, -1)
        for z in range(n):
            mz = z if z <= n // 2 else z - n
            for q in range(K1):
                res[z, :, q] = spectral(res[z, :, q], q, myp - K, mz, K, op_curl)
        out_z = fft_batch(res, logn, twi, +1)
        B[:, myp] = np.moveaxis(out_z, 0, 1)
    # y inverse (zero padded) -> A[c][z][y][kx]
    for c in range(3):
        for z in range(n):
            buf = np.zeros((n, K1), complex)
            for y in range(n):
                my = y if y <= n // 2 else y - n
                if -K <= my <= K:
                    buf[y] = B[c, my + K, z]
            A[c, z] = fft_batch(buf, logn, twi, +1)
    # x inverse: Hermitian completion, real part
    out = np.empty_like(g)
    for c in range(3):
        for z in range(n):
            buf = np.zeros((n, n), complex)                # [m][y]
            for m in range(n):
                if m < K1:
                    buf[m] = A[c, z, :, m]
                elif n - m < K1:
                    buf[m] = np.conj(A[c, z, :, n - m])
            out[c, z] = fft_batch(buf, logn, twi, +1).real.T
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
