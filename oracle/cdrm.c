/*
 * Oracle DRM entries in plain C (test infrastructure; never linked into the product).
 *
 * The same definition as oracle/drm.py, G(seed, node, kind, row, col), evaluated by the
 * same sequence of correctly rounded binary64 operations, so that the two agree bit for
 * bit (pinned by tests/test_oracle_drm.py):
 *   Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) on counter (lo32 row, hi32 row,
 *   col, tag = 2 node + kind) and key (lo32 seed, hi32 seed);
 *   u1 = (a + 1) 2^-53, u2 = b 2^-53 from the high 53 bits of (x1:x0) and (x3:x2);
 *   z = sqrt(-2 ln u1) cos(2 pi u2), ln by the atanh series, cos(2 pi .) by Taylor
 *   series after exact reduction to [0, 1/4].
 * Build with -ffp-contract=off (no fused multiply-add) and without fast-math.
 */
#include <math.h>
#include <stdint.h>

static void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    const uint32_t n3 = (uint32_t)p0;
    c[0] = n0;
    c[1] = n1;
    c[2] = n2;
    c[3] = n3;
  }
}

static double LNC[24], COSC[11], SINC[11];
static double SQRT2, LN2, TWOPI;
static int ready = 0;

static void init(void) {
  if (ready) return;
  for (int k = 3; k < 24; k += 2) LNC[k] = 1.0 / (double)k;
  COSC[0] = 1.0;
  SINC[0] = 1.0;
  for (int k = 1; k <= 10; ++k) {
    COSC[k] = -COSC[k - 1] / (double)((2 * k - 1) * (2 * k));
    SINC[k] = -SINC[k - 1] / (double)((2 * k) * (2 * k + 1));
  }
  SQRT2 = 0x1.6a09e667f3bcdp+0;
  LN2 = 0x1.62e42fefa39efp-1;
  TWOPI = 0x1.921fb54442d18p+2;
  ready = 1;
}

static double ln_fixed(double u) {
  int E;
  const double m = frexp(u, &E);   /* u = m 2^E, m in [0.5, 1) */
  double f = m * 2.0;
  double e = (double)(E - 1);
  if (f > SQRT2) {
    f = f * 0.5;
    e = e + 1.0;
  }
  const double s = (f - 1.0) / (f + 1.0);
  const double w = s * s;
  double P = LNC[23];
  for (int k = 21; k > 2; k -= 2) P = LNC[k] + w * P;
  const double lnf = 2.0 * (s + s * (w * P));
  return e * LN2 + lnf;
}

static double horner(double y, const double* c) {
  double acc = c[10];
  for (int k = 9; k >= 0; --k) acc = c[k] + y * acc;
  return acc;
}

static double cos2pi_fixed(double v) {
  if (v >= 0.5) v = 1.0 - v;
  double sg = 1.0;
  if (v > 0.25) {
    v = 0.5 - v;
    sg = -1.0;
  }
  double c;
  if (v <= 0.125) {
    const double x = TWOPI * v;
    c = horner(x * x, COSC);
  } else {
    const double x = TWOPI * (0.25 - v);
    c = x * horner(x * x, SINC);
  }
  return sg * c;
}

static double gauss(uint64_t seed, uint32_t tag, uint64_t row, uint32_t col) {
  uint32_t c[4] = {(uint32_t)row, (uint32_t)(row >> 32), col, tag};
  philox(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t a = ((((uint64_t)c[1]) << 32) | c[0]) >> 11;
  const uint64_t b = ((((uint64_t)c[3]) << 32) | c[2]) >> 11;
  const double u1 = (double)(a + 1) * 0x1p-53;
  const double u2 = (double)b * 0x1p-53;
  return sqrt(-2.0 * ln_fixed(u1)) * cos2pi_fixed(u2);
}

/* out[i] = G(seed, tag, rows[i], cols[i]) for i < n. */
void oracle_gaussian(uint64_t seed, uint32_t tag, const uint64_t* rows, const uint32_t* cols, int64_t n,
                     double* out) {
  init();
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = gauss(seed, tag, rows[i], cols[i]);
}

/* Dense rows row0 .. row0 + nrows - 1 of a DRM with ncols columns, row-major. */
void oracle_drm_rows(uint64_t seed, uint32_t tag, int64_t row0, int64_t nrows, int64_t ncols, double* out) {
  init();
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < nrows; ++r)
    for (int64_t c = 0; c < ncols; ++c) out[r * ncols + c] = gauss(seed, tag, (uint64_t)(row0 + r), (uint32_t)c);
}
