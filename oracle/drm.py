"""Seeded Gaussian dimension-reduction maps of the oracle (test infrastructure).

The paper only asks for standard Gaussian DRMs (Sec. 4, eq. "sketch"; Lemma 4 and
Theorem 2 assume i.i.d. N(0,1) entries).  Entry (row, col) of the DRM of kind
`kind` (0 = right map X_t, 1 = left map Y_t) of node `node` (level-order id) is a
pure function G(seed, node, kind, row, col):

  1. Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel random
     numbers: as easy as 1, 2, 3", SC'11) on counter
     (lo32(row), hi32(row), col, 2*node + kind) and key (lo32(seed), hi32(seed)).
  2. Two 53-bit uniforms u1 = (a + 1) 2^-53 in (0, 1] and u2 = b 2^-53 in [0, 1)
     from the high 53 bits of the 64-bit words (x1:x0) and (x3:x2).
  3. Box-Muller, z = sqrt(-2 ln u1) cos(2 pi u2), where ln and cos(2 pi .) are
     evaluated by the fixed sequences of correctly rounded binary64 operations
     below (an atanh series for ln, Taylor series after exact argument
     reduction for the cosine), so that any IEEE-conforming implementation
     produces the same bits.
  4. Reduced copies: fp32 = round-to-nearest(z); bf16 = round-to-nearest-even of
     the fp32 bit pattern to its upper 16 bits.

NumPy float64 ufuncs perform each operation with a single IEEE rounding and never
fuse a multiply with an add, which is what the bit-for-bit definition needs.
"""

import numpy as np

# Philox4x32 constants as published in the SC'11 paper.
_PHILOX_M0 = np.uint64(0xD2511F53)
_PHILOX_M1 = np.uint64(0xCD9E8D57)
_PHILOX_W0 = 0x9E3779B9
_PHILOX_W1 = 0xBB67AE85
_MASK32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

# doubles nearest to the named reals (hex literals, exact)
SQRT2 = float.fromhex("0x1.6a09e667f3bcdp+0")
LN2 = float.fromhex("0x1.62e42fefa39efp-1")
TWOPI = float.fromhex("0x1.921fb54442d18p+2")
TWO_M53 = float.fromhex("0x1p-53")


def philox4x32_10(ctr, key):
    """Philox4x32-10 on arrays.  ctr: 4 arrays of 32-bit values, key: 2 ints."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & _MASK32 for c in ctr)
    k0 = int(key[0]) & 0xFFFFFFFF
    k1 = int(key[1]) & 0xFFFFFFFF
    for rnd in range(10):
        if rnd:
            k0 = (k0 + _PHILOX_W0) & 0xFFFFFFFF
            k1 = (k1 + _PHILOX_W1) & 0xFFFFFFFF
        p0 = _PHILOX_M0 * c0          # exact: product of two 32-bit values fits 64 bits
        p1 = _PHILOX_M1 * c2
        hi0, lo0 = p0 >> _S32, p0 & _MASK32
        hi1, lo1 = p1 >> _S32, p1 & _MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
    return c0, c1, c2, c3


def _ln_coeffs():
    return {k: 1.0 / k for k in range(3, 24, 2)}


_LNC = _ln_coeffs()


def ln_fixed(u):
    """Natural log for u in (0, 1] by the atanh series (fixed operation order)."""
    u = np.asarray(u, dtype=np.float64)
    m, E = np.frexp(u)                      # u = m 2^E, m in [0.5, 1)
    f = m * 2.0                             # exact, f in [1, 2)
    e = (E - 1).astype(np.float64)
    big = f > SQRT2
    f = np.where(big, f * 0.5, f)           # exact
    e = np.where(big, e + 1.0, e)
    s = (f - 1.0) / (f + 1.0)
    w = s * s
    P = np.full_like(s, _LNC[23])
    for k in range(21, 2, -2):
        P = _LNC[k] + w * P
    lnf = 2.0 * (s + s * (w * P))
    return e * LN2 + lnf


def _cos_coeffs():
    a = [1.0]
    for k in range(1, 11):
        a.append(-a[-1] / float((2 * k - 1) * (2 * k)))
    return a


def _sin_coeffs():
    b = [1.0]
    for k in range(1, 11):
        b.append(-b[-1] / float((2 * k) * (2 * k + 1)))
    return b


_COSC = _cos_coeffs()
_SINC = _sin_coeffs()


def _horner(y, coeffs):
    c = np.full_like(y, coeffs[-1])
    for a in reversed(coeffs[:-1]):
        c = a + y * c
    return c


def cos2pi_fixed(v):
    """cos(2 pi v) for v in [0, 1) after exact reduction to [0, 1/4]."""
    v = np.asarray(v, dtype=np.float64)
    v = np.where(v >= 0.5, 1.0 - v, v)      # exact (Sterbenz)
    neg = v > 0.25
    v = np.where(neg, 0.5 - v, v)           # exact
    sg = np.where(neg, -1.0, 1.0)
    xc = TWOPI * v
    cser = _horner(xc * xc, _COSC)
    xs = TWOPI * (0.25 - v)                 # 0.25 - v exact on (1/8, 1/4]
    sser = xs * _horner(xs * xs, _SINC)
    c = np.where(v <= 0.125, cser, sser)
    return sg * c


def gaussian(seed, node, kind, rows, cols):
    """G(seed, node, kind, row, col) as float64 for broadcastable index arrays.  Uses
    the plain-C evaluation of the same definition (oracle/cdrm.c, bit-identical) when
    it is built, else gaussian_numpy."""
    from . import cdrm
    if cdrm.lib() is not None:
        rows, cols = np.broadcast_arrays(np.asarray(rows, dtype=np.uint64), np.asarray(cols, dtype=np.uint64))
        out = cdrm.gaussian(seed, 2 * node + kind, rows.ravel(), cols.ravel().astype(np.uint32))
        return out.reshape(rows.shape)
    return gaussian_numpy(seed, node, kind, rows, cols)


def gaussian_numpy(seed, node, kind, rows, cols):
    """The definition of G in NumPy float64 operations (the reference the C
    evaluation is pinned to)."""
    rows = np.asarray(rows, dtype=np.uint64)
    cols = np.asarray(cols, dtype=np.uint64)
    rows, cols = np.broadcast_arrays(rows, cols)
    seed = int(seed)
    ctr = (rows & _MASK32, rows >> _S32, cols, np.full(rows.shape, 2 * node + kind, np.uint64))
    x0, x1, x2, x3 = philox4x32_10(ctr, (seed & 0xFFFFFFFF, seed >> 32))
    a = ((x1 << _S32) | x0) >> np.uint64(11)
    b = ((x3 << _S32) | x2) >> np.uint64(11)
    u1 = (a + np.uint64(1)).astype(np.float64) * TWO_M53
    u2 = b.astype(np.float64) * TWO_M53
    return np.sqrt(-2.0 * ln_fixed(u1)) * cos2pi_fixed(u2)


def drm(seed, node, kind, nrows, ncols, chunk=1 << 22):
    """Dense DRM of shape (nrows, ncols), float64, generated in row chunks."""
    from . import cdrm
    if cdrm.lib() is not None:
        return cdrm.drm_rows(seed, 2 * node + kind, 0, nrows, ncols)
    out = np.empty((nrows, ncols), dtype=np.float64)
    step = max(1, chunk // max(1, ncols))
    cols = np.arange(ncols, dtype=np.uint64)[None, :]
    for r0 in range(0, nrows, step):
        r1 = min(nrows, r0 + step)
        rows = np.arange(r0, r1, dtype=np.uint64)[:, None]
        out[r0:r1] = gaussian(seed, node, kind, rows, cols)
    return out


def to_fp32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def bf16_bits(x):
    """bf16 bit patterns (uint16) of round-to-nearest-even of fp32(x)."""
    b = to_fp32(x).view(np.uint32).astype(np.uint64)
    return ((b + np.uint64(0x7FFF) + ((b >> np.uint64(16)) & np.uint64(1))) >> np.uint64(16)).astype(np.uint16)


def bf16_to_f64(bits):
    return (np.asarray(bits, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)


def rounded(x, dtype):
    """Value of x after storage in `dtype` ('f64', 'f32', 'bf16'), as float64."""
    if dtype == "f64":
        return np.asarray(x, dtype=np.float64)
    if dtype == "f32":
        return to_fp32(x).astype(np.float64)
    if dtype == "bf16":
        return bf16_to_f64(bf16_bits(x))
    raise ValueError(dtype)
