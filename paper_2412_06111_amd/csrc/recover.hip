// Recovery-phase linear algebra in FP64 on the GPU (Sec. 4 "Recovery phase",
// Alg. 2, stabilised least squares with eps = eps_factor * ||R||_2), one workgroup
// per tree node:
//   1. Householder QR of Omega_t (k x r, k >= r), reflectors kept in LDS;
//      Q = H_0 ... H_{r-1} [I; 0];  signs flipped so that diag(R) >= 0.
//   2. One-sided (Hestenes) Jacobi SVD of the r x r factor R, applied to R^T: column
//      pairs of R^T are rotated in round-robin order until every pair is orthogonal to
//      working precision; sigma_p = ||w_p||, V accumulates the rotations.
//   3. R^{+eps} = sum_{sigma_p > eps} v_p u_p^T / sigma_p with eps = eps_factor * max sigma.
//   When ||R||_F ||R^{-1}||_F < 1/(2 eps_factor) no singular value can fall below
//   eps, so R^{+eps} = R^{-1} is formed by back substitution and the SVD is skipped.
// Also: deterministic squared-norm reductions used for error reporting.
#include <algorithm>
#include <mutex>

#include "kernels.hpp"

namespace ttnn {
namespace {

constexpr int kThreads = 256;


// DPP move of a double (both halves); lanes whose source is out of the row pattern or
// outside row_mask read 0
template <int CTRL, int ROW_MASK = 0xF>
__device__ inline double dpp64(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int lo2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROW_MASK, 0xF, false);
  const int hi2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROW_MASK, 0xF, false);
  return __hiloint2double(hi2, lo2);
}

// 8 lanes per matrix column: the sum over the group of 8 consecutive lanes, in every
// lane of the group (quad sums, then the mirrored quad of the half row; a + b = b + a
// exactly, so all lanes agree)
__device__ inline double group8_sum(double v) {
  v += dpp64<0xB1>(v);            // quad_perm [1,0,3,2]
  v += dpp64<0x4E>(v);            // quad_perm [2,3,0,1]
  v += dpp64<0x141>(v);           // row_half_mirror: lane i <-> 7 - i
  return v;
}

// Sum over the 64 lanes of a wave in a fixed order, returned to every lane: row sums
// by DPP, rows combined by row broadcasts into lane 63, then read from lane 63.
// The same over groups of 4 consecutive lanes (quad sums).
__device__ inline double group4_sum(double v) {
  v += dpp64<0xB1>(v);            // quad_perm [1,0,3,2]
  v += dpp64<0x4E>(v);            // quad_perm [2,3,0,1]
  return v;
}

template <int LPC>
__device__ inline double group_sum(double v) {
  static_assert(LPC == 4 || LPC == 8, "4 or 8 lanes per column");
  return LPC == 8 ? group8_sum(v) : group4_sum(v);
}

__device__ inline double wave_sum64(double v) {
  v += dpp64<0xB1>(v);
  v += dpp64<0x4E>(v);
  v += dpp64<0x141>(v);           // half-row sums
  v += dpp64<0x140>(v);           // row_mirror: row sums in every lane of the row
  v += dpp64<0x142, 0xA>(v);      // row_bcast:15 into rows 1 and 3
  v += dpp64<0x143, 0xC>(v);      // row_bcast:31 into rows 2 and 3: lane 63 holds the total
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

__device__ inline double block_sum(double v, double* red) {
  // 256 threads: wave reduction then across the 4 waves
  v = wave_sum64(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  const double s = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  return s;
}

// Apply H_j = I - tau v v^T (v_j = 1, v_i = A[i + ld j] for i > j) to columns
// [c0, c1) of the k-row column-major matrix X (leading dimension ld).
__device__ inline void apply_reflector(const double* A, int ld, int k, int j, double tau, double* X, int c0, int c1) {
  const int g = threadIdx.x >> 3, sub = threadIdx.x & 7;
  for (int cbase = c0; cbase < c1; cbase += kThreads / 8) {
    const int c = cbase + g;
    const bool on = c < c1;
    double w = 0.0;
    if (on)
      for (int i = j + sub; i < k; i += 8) w += (i == j ? 1.0 : A[i + ld * j]) * X[i + ld * c];
    w = group8_sum(w) * tau;
    if (on)
      for (int i = j + sub; i < k; i += 8) X[i + ld * c] -= w * (i == j ? 1.0 : A[i + ld * j]);
  }
}

// ---------------------------------------------------------------- register path
// r <= 256 / LPC and k <= LPC TM: column c of Omega lives in the registers of the LPC
// lanes tid = LPC c .. LPC c + LPC - 1 (lane sub holds rows sub + LPC t, t < TM); 8
// lanes per column up to r = 32, 4 up to r = 64.  A factorization step
// forms the reflector in its column's lanes, broadcasts it through LDS (double
// buffered) and takes one barrier; every other column applies it in registers.  Q and
// R^{-1} are then formed column by column from reflectors and R in LDS, with no
// barrier.  Returns true on the fast path (Q, Pinv = R^{-1}, kept written); otherwise
// leaves R in W and the identity in V (leading dimension r) for the Jacobi path.
template <int TM, int LPC>
__device__ bool qr_regs(const QrJob& job, double eps_factor, double* A, int ld, double* W, double* V,
                        double* vb, double* tau_s, double* red, int* kept) {
  const int k = job.k, r = job.r;
  const int tid = threadIdx.x, c = tid / LPC, sub = tid % LPC;
  const bool own = c < r;
  double a[TM];
#pragma unroll
  for (int t = 0; t < TM; ++t) {
    const int i = sub + LPC * t;
    a[t] = (own && i < k) ? job.Om[i + static_cast<int64_t>(k) * c] : 0.0;
  }
  // ---- factorization (LAPACK dlarfg convention, v_j = 1)
  for (int j = 0; j < r; ++j) {
    double* vj = vb + (j & 1) * LPC * TM;
    if (c == j) {
      double n0 = 0.0, n1 = 0.0, al = 0.0;
#pragma unroll
      for (int t = 0; t < TM; ++t) {
        const int i = sub + LPC * t;
        const double x = i > j ? a[t] : 0.0;
        if (t & 1) n1 = fma(x, x, n1);
        else n0 = fma(x, x, n0);
        al += i == j ? a[t] : 0.0;
      }
      const double xnorm2 = group_sum<LPC>(n0 + n1);
      const double alpha = group_sum<LPC>(al);
      double tau = 0.0, beta = alpha, scale = 0.0;
      if (xnorm2 > 0.0) {
        beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
#pragma unroll
      for (int t = 0; t < TM; ++t) {
        const int i = sub + LPC * t;
        const double v = i > j ? a[t] * scale : (i == j ? 1.0 : 0.0);
        vj[i] = v;
        a[t] = i > j ? v : (i == j ? beta : a[t]);
      }
      if (sub == 0) tau_s[j] = tau;
    }
    __syncthreads();
    if (own && c > j) {
      const double tau = tau_s[j];
      if (tau != 0.0) {
        double v[TM];
        double w0 = 0.0, w1 = 0.0;
#pragma unroll
        for (int t = 0; t < TM; ++t) {
          v[t] = vj[sub + LPC * t];
          if (t & 1) w1 = fma(v[t], a[t], w1);
          else w0 = fma(v[t], a[t], w0);
        }
        const double w = group_sum<LPC>(w0 + w1) * tau;
#pragma unroll
        for (int t = 0; t < TM; ++t) a[t] = fma(-w, v[t], a[t]);
      }
    }
  }
  // reflectors and R to LDS (column c: R on and above the diagonal, v below)
  if (own) {
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      const int i = sub + LPC * t;
      if (i < k) A[i + ld * c] = a[t];
    }
  }
  __syncthreads();
  // ---- Q = H_0 ... H_{r-1} [I; 0], column by column (H_j e_c = e_c for j > c exactly)
  const double rcc = own ? A[c + ld * c] : 1.0;
  const double sgn = rcc < 0.0 ? -1.0 : 1.0;
  {
    double q[TM];
#pragma unroll
    for (int t = 0; t < TM; ++t) q[t] = (sub + LPC * t) == c ? 1.0 : 0.0;
    for (int j = r - 1; j >= 0; --j) {
      const double tau = tau_s[j];
      if (tau == 0.0) continue;
      double v[TM];
      double w0 = 0.0, w1 = 0.0;
#pragma unroll
      for (int t = 0; t < TM; ++t) {
        const int i = sub + LPC * t;
        v[t] = i > j ? (i < k ? A[i + ld * j] : 0.0) : (i == j ? 1.0 : 0.0);
        if (t & 1) w1 = fma(v[t], q[t], w1);
        else w0 = fma(v[t], q[t], w0);
      }
      const double w = group_sum<LPC>(w0 + w1) * tau;
#pragma unroll
      for (int t = 0; t < TM; ++t) q[t] = fma(-w, v[t], q[t]);
    }
    if (own) {
#pragma unroll
      for (int t = 0; t < TM; ++t) {
        const int i = sub + LPC * t;
        if (i < k) job.Q[i + static_cast<int64_t>(k) * c] = sgn * q[t];
      }
    }
  }
  // ---- W = diag(sign R(i, i)) R, upper triangular (leading dimension r) in registers and LDS
  double w[TM];
  double wn = 0.0;
#pragma unroll
  for (int t = 0; t < TM; ++t) {
    const int i = sub + LPC * t;
    double x = 0.0;
    if (own && i <= c) x = A[i + ld * i] < 0.0 ? -a[t] : a[t];
    w[t] = x;
    wn = fma(x, x, wn);
  }
  __syncthreads();                        // A (the reflectors) is read; W and V may overwrite it
  if (own) {
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      const int i = sub + LPC * t;
      if (i < r) W[i + r * c] = w[t];
    }
  }
  const double rnorm2 = block_sum(wn, red);   // its barriers also publish W
  // ---- V = W^{-1} column by column: x = W^{-1} e_c, m = r-1 .. 0
  double x[TM];
#pragma unroll
  for (int t = 0; t < TM; ++t) x[t] = (sub + LPC * t) == c ? 1.0 : 0.0;
  bool nonsingular = true;
  for (int m = r - 1; m >= 0; --m) {
    const double dm = W[m + r * m];
    nonsingular = nonsingular && dm > 0.0;
    double xl = 0.0;
#pragma unroll
    for (int t = 0; t < TM; ++t) xl += (sub + LPC * t) == m ? x[t] : 0.0;
    const double xm = group_sum<LPC>(xl) / dm;
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      const int i = sub + LPC * t;
      const double wim = i < m ? W[i + r * m] : 0.0;
      x[t] = i == m ? xm : (i < m ? fma(-xm, wim, x[t]) : x[t]);
    }
  }
  double vn = 0.0;
#pragma unroll
  for (int t = 0; t < TM; ++t) vn += (own && (sub + LPC * t) < r) ? x[t] * x[t] : 0.0;
  const double inv2 = block_sum(vn, red);
  const bool fast = nonsingular && (sqrt(rnorm2 * inv2) * eps_factor < 0.5);
  if (fast) {
    if (own) {
#pragma unroll
      for (int t = 0; t < TM; ++t) {
        const int i = sub + LPC * t;
        if (i < r) job.Pinv[i + r * c] = x[t];
      }
    }
    if (tid == 0) kept[job.slot] = r;
    return true;
  }
  for (int e = tid; e < r * r; e += kThreads) V[e] = ((e % r) == (e / r)) ? 1.0 : 0.0;
  __syncthreads();
  return false;
}

// WTM: 0 for the narrow register paths (r <= 32) and the LDS path; 16 or 24 for the
// jobs with 32 < r <= 64 and k <= 64 or k <= 96 (4 lanes per column, WTM rows a lane).
// Each form is an instance of its own so that its register demand does not lower the
// occupancy of the others.
constexpr int kQrMaxR = 128;   // columns of the per-column arrays below
// static LDS of qr_pinv_kernel: red, tau_s, sig, vb (doubles) and two flags
constexpr size_t kQrStaticLds = sizeof(double) * (4 + kQrMaxR + kQrMaxR + 2 * kQrMaxR) + 2 * sizeof(int);
constexpr size_t kLdsPerWorkgroup = 160 * 1024;

template <int WTM>
__global__ __launch_bounds__(kThreads) void qr_pinv_kernel(QrJobList jl, double eps_factor, int* kept) {
  extern __shared__ double lds[];
  __shared__ double red[4];
  __shared__ double tau_s[kQrMaxR];
  __shared__ double sig[kQrMaxR];
  __shared__ int any_rot;
  __shared__ int fast;
  const QrJob job = jl.jobs[blockIdx.x];
  const int k = job.k, r = job.r;
  const int tid = threadIdx.x;
  const int ld = k | 1;          // odd leading dimension: the 8 columns a wave touches at once spread over the banks
  double* A = lds;               // ld x r: Omega, then reflectors below the diagonal and R above
  double* Qm = A + ld * r;       // ld x r: Q
  double* W = Qm;                // r x r (after Q is stored): R, then the Jacobi columns
  double* V = A;                 // r x r (after R is extracted): R^{-1}, or right singular vectors

  __shared__ double vb[2 * kQrMaxR];
  // register path: 8 lanes per column for r <= 32 (k <= 128), 4 for r <= 64 (k <= 64)
  const int tm = WTM ? WTM : r <= 32 ? (k <= 32 ? 4 : k <= 48 ? 6 : k <= 64 ? 8 : k <= 128 ? 16 : 0) : 0;
  if (tm != 0) {
    const bool f = WTM        ? qr_regs<(WTM ? WTM : 16), 4>(job, eps_factor, A, ld, W, V, vb, tau_s, red, kept)
                   : tm == 4  ? qr_regs<4, 8>(job, eps_factor, A, ld, W, V, vb, tau_s, red, kept)
                   : tm == 6  ? qr_regs<6, 8>(job, eps_factor, A, ld, W, V, vb, tau_s, red, kept)
                   : tm == 8  ? qr_regs<8, 8>(job, eps_factor, A, ld, W, V, vb, tau_s, red, kept)
                              : qr_regs<16, 8>(job, eps_factor, A, ld, W, V, vb, tau_s, red, kept);
    if (f) return;
  } else {
  for (int e = tid; e < k * r; e += kThreads) A[e % k + ld * (e / k)] = job.Om[e];
  __syncthreads();

  // ---- Householder QR (LAPACK dlarfg convention, v_0 = 1).  Wave 0 forms each
  // reflector with shuffles (rows strided over its 64 lanes, fixed order); all
  // threads apply it to the remaining columns; two barriers per column.
  for (int j = 0; j < r; ++j) {
    if (tid < 64) {
      double part = 0.0;
      for (int i = j + 1 + tid; i < k; i += 64) part += A[i + ld * j] * A[i + ld * j];
      const double xnorm2 = wave_sum64(part);
      const double alpha = A[j + ld * j];
      double tau = 0.0, beta = alpha, scale = 0.0;
      if (xnorm2 > 0.0) {
        beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
        for (int i = j + 1 + tid; i < k; i += 64) A[i + ld * j] *= scale;
      }
      if (tid == 0) {
        A[j + ld * j] = beta;
        tau_s[j] = tau;
      }
    }
    __syncthreads();
    const double tau = tau_s[j];
    if (tau != 0.0) apply_reflector(A, ld, k, j, tau, A, j + 1, r);
    __syncthreads();
  }

  // ---- Q = H_0 ... H_{r-1} [I; 0]
  for (int e = tid; e < k * r; e += kThreads) Qm[e % k + ld * (e / k)] = ((e % k) == (e / k)) ? 1.0 : 0.0;
  __syncthreads();
  for (int j = r - 1; j >= 0; --j) {
    const double tau = tau_s[j];
    if (tau != 0.0) apply_reflector(A, ld, k, j, tau, Qm, j, r);
    __syncthreads();
  }
  // sign fix diag(R) >= 0: flip row j of R and column j of Q
  for (int e = tid; e < k * r; e += kThreads) {
    const int c = e / k;
    const double v = Qm[e % k + ld * c];
    job.Q[e] = (A[c + ld * c] < 0.0) ? -v : v;
  }
  __syncthreads();
  for (int e = tid; e < r * r; e += kThreads) {
    const int i = e % r, c = e / r;
    double v = (i <= c) ? A[i + ld * c] : 0.0;
    if (A[i + ld * i] < 0.0) v = -v;
    W[e] = v;
  }
  __syncthreads();

  // ---- fast path: if ||R||_F ||R^{-1}||_F < 1 / (2 eps_factor) then sigma_min / sigma_max
  // exceeds eps_factor, nothing is truncated and R^{+eps} = R^{-1} (back substitution)
  {
    double part = 0.0;
    for (int e = tid; e < r * r; e += kThreads) part += W[e] * W[e];
    const double rnorm2 = block_sum(part, red);
    bool nonsingular = true;
    for (int i = 0; i < r; ++i) nonsingular = nonsingular && (W[i + r * i] > 0.0);
    double inv2 = 0.0;
    if (nonsingular) {
      // R^{-1} by back substitution, row i = r-1 .. 0 for all columns at once:
      // V[i][c] = (delta_ic - sum_{i<m<=c} R[i][m] V[m][c]) / R[i][i], 8 lanes per column
      for (int e = tid; e < r * r; e += kThreads) V[e] = 0.0;
      __syncthreads();
      const int g = tid >> 3, sub = tid & 7;
      for (int i = r - 1; i >= 0; --i) {
        for (int cbase = i; cbase < r; cbase += kThreads / 8) {
          const int c = cbase + g;
          double sacc = 0.0;
          if (c < r)
            for (int m = i + 1 + sub; m <= c; m += 8) sacc += W[i + r * m] * V[m + r * c];
          sacc = group8_sum(sacc);
          if (c < r && sub == 0) V[i + r * c] = ((i == c ? 1.0 : 0.0) - sacc) / W[i + r * i];
        }
        __syncthreads();
      }
      for (int e = tid; e < r * r; e += kThreads) inv2 += V[e] * V[e];
    }
    inv2 = block_sum(inv2, red);
    if (tid == 0) fast = nonsingular && (sqrt(rnorm2 * inv2) * eps_factor < 0.5);
    __syncthreads();
    if (fast) {
      for (int e = tid; e < r * r; e += kThreads) job.Pinv[e] = V[e];
      if (tid == 0) kept[job.slot] = r;
      return;
    }
  }
  for (int e = tid; e < r * r; e += kThreads) V[e] = ((e % r) == (e / r)) ? 1.0 : 0.0;
  __syncthreads();
  }

  // ---- one-sided Jacobi on the columns of W = R^T (the rows of R): on the graded,
  // ill-conditioned triangular factors of these sketches the rows converge in about 10
  // sweeps where the columns take 25 (the preconditioning effect of the QR that
  // Drmac and Veselic describe for one-sided Jacobi).  W V = U S with V orthogonal gives
  // R = V S U^T, so R^+ = U S^-1 V^T = sum_p w_p v_p^T / s_p^2.  A pair is rotated while
  // its cosine exceeds twice the rounding bound r u of the length-r dot product that
  // measures it (u = 2^-53).
  for (int e = tid; e < r * r; e += kThreads) {
    const int i = e % r, c = e / r;
    if (i < c) {
      const double t = W[i + r * c];
      W[i + r * c] = W[c + r * i];
      W[c + r * i] = t;
    }
  }
  __syncthreads();
  const int R2 = r + (r & 1);                 // pad to even with a virtual zero column
  const int npairs = R2 / 2;
  const double jtol = fmax(1e-15, r * 0x1p-52);
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) any_rot = 0;
    __syncthreads();
    for (int step = 0; step < R2 - 1; ++step) {
      // round-robin pairing: player 0 fixed, the others rotate
      for (int pr = tid / 8; pr < npairs; pr += kThreads / 8) {
        const int lane8 = tid % 8;
        auto player = [&](int pos) { return pos == 0 ? 0 : 1 + ((pos - 1 + step) % (R2 - 1)); };
        int p = player(pr), q = player(R2 - 1 - pr);
        if (p > q) { const int t = p; p = q; q = t; }
        double al = 0.0, be = 0.0, ga = 0.0;
        if (q < r) {
          for (int i = lane8; i < r; i += 8) {
            const double x = W[i + r * p], y = W[i + r * q];
            al += x * x;
            be += y * y;
            ga += x * y;
          }
        }
        al = group8_sum(al);
        be = group8_sum(be);
        ga = group8_sum(ga);
        if (q < r && ga != 0.0 && fabs(ga) > jtol * sqrt(al * be)) {
          const double zeta = (be - al) / (2.0 * ga);
          const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + t * t);
          const double sn = cs * t;
          for (int i = lane8; i < r; i += 8) {
            const double x = W[i + r * p], y = W[i + r * q];
            W[i + r * p] = cs * x - sn * y;
            W[i + r * q] = sn * x + cs * y;
            const double vx = V[i + r * p], vy = V[i + r * q];
            V[i + r * p] = cs * vx - sn * vy;
            V[i + r * q] = sn * vx + cs * vy;
          }
          if (lane8 == 0) any_rot = 1;
        }
      }
      __syncthreads();
    }
    const int rot = any_rot;
    __syncthreads();
    if (!rot) break;
  }

  // ---- singular values and truncated pseudo-inverse
  for (int c = tid; c < r; c += kThreads) {
    double s = 0.0;
    for (int i = 0; i < r; ++i) s += W[i + r * c] * W[i + r * c];
    sig[c] = sqrt(s);
  }
  __syncthreads();
  double smax = 0.0;
  for (int c = 0; c < r; ++c) smax = fmax(smax, sig[c]);
  const double eps = eps_factor * smax;
  for (int e = tid; e < r * r; e += kThreads) {
    const int i = e % r, j = e / r;            // Pinv(i, j) = sum_p W(i,p) V(j,p) / sigma_p^2
    double s = 0.0;
    for (int p = 0; p < r; ++p)
      if (sig[p] > eps) s += W[i + r * p] * V[j + r * p] / (sig[p] * sig[p]);
    job.Pinv[e] = s;
  }
  if (tid == 0) {
    int cnt = 0;
    for (int p = 0; p < r; ++p) cnt += sig[p] > eps ? 1 : 0;
    kept[job.slot] = cnt;
  }
}

// one thread: an assembly is bad if a sketch was not finite or a node kept nothing
__global__ void status_fold_kernel(const int* __restrict__ flags, int nn, int* __restrict__ call,
                                   int* __restrict__ sticky) {
  if (threadIdx.x != 0) return;
  int bad = flags[0] != 0 ? 1 : 0;
  for (int v = 1; v < nn; ++v) bad |= flags[v] == 0 ? 1 : 0;
  *call = bad;
  *sticky = *sticky | bad;
}

__global__ void diff_norm_part(const void* a, int a_dtype, const double* b, int64_t n, double* part) {
  double s0 = 0.0, s1 = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    double av;
    if (a_dtype == TTNN_F64) av = static_cast<const double*>(a)[i];
    else if (a_dtype == TTNN_F32) av = static_cast<const float*>(a)[i];
    else av = bf16_bits_to_f32(static_cast<const uint16_t*>(a)[i]);
    const double bv = b[i];
    s0 += (av - bv) * (av - bv);
    s1 += bv * bv;
  }
  __shared__ double red[4];
  s0 = block_sum(s0, red);
  s1 = block_sum(s1, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s0;
    part[2 * blockIdx.x + 1] = s1;
  }
}

__global__ void diff_norm_final(const double* part, int nb, double* out) {
  if (threadIdx.x == 0) {
    double s0 = 0.0, s1 = 0.0;
    for (int i = 0; i < nb; ++i) {
      s0 += part[2 * i];
      s1 += part[2 * i + 1];
    }
    out[0] = s0;
    out[1] = s1;
  }
}

}  // namespace

size_t qr_pinv_lds_bytes(int k, int r) { return static_cast<size_t>(2 * (k | 1)) * r * sizeof(double); }

bool qr_pinv_fits(int k, int r) {
  return k >= r && r >= 1 && r <= kQrMaxR && k <= 2 * kQrMaxR &&
         qr_pinv_lds_bytes(k, r) + kQrStaticLds <= kLdsPerWorkgroup;
}

void launch_qr_pinv(const QrJobList& jl, double eps_factor, int* d_kept, hipStream_t st) {
  if (jl.n <= 0) return;
  QrJobList lists[3] = {};
  size_t need[3] = {0, 0, 0};                 // dynamic LDS of each launch: its largest job
  for (int i = 0; i < jl.n; ++i) {
    const QrJob& j = jl.jobs[i];
    if (!qr_pinv_fits(j.k, j.r))
      throw Error{TTNN_E_INVALID, "recovery job k = " + std::to_string(j.k) + ", r = " + std::to_string(j.r) +
                                      " exceeds one workgroup's LDS"};
    const int w = (j.r > 32 && j.r <= 64) ? (j.k <= 64 ? 1 : j.k <= 96 ? 2 : 0) : 0;
    lists[w].jobs[lists[w].n++] = j;
    need[w] = std::max(need[w], qr_pinv_lds_bytes(j.k, j.r));
  }
  auto launch = [&](const void* fn, int w, void (*k)(QrJobList, double, int*)) {
    const QrJobList& l = lists[w];
    if (l.n == 0) return;
    const size_t lds = need[w];
    if (lds > 64 * 1024) {
      const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
      if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error{TTNN_E_INVALID, "recovery kernel needs " + std::to_string(lds) + " bytes of LDS"};
      }
    }
    hipLaunchKernelGGL(k, dim3(l.n), dim3(kThreads), lds, st, l, eps_factor, d_kept);
  };
  launch(reinterpret_cast<const void*>(qr_pinv_kernel<0>), 0, qr_pinv_kernel<0>);
  launch(reinterpret_cast<const void*>(qr_pinv_kernel<16>), 1, qr_pinv_kernel<16>);
  launch(reinterpret_cast<const void*>(qr_pinv_kernel<24>), 2, qr_pinv_kernel<24>);
}

void launch_status_fold(const int* flags, int nn, int* call, int* sticky, hipStream_t st) {
  hipLaunchKernelGGL(status_fold_kernel, dim3(1), dim3(64), 0, st, flags, nn, call, sticky);
}

void launch_diff_norms(const void* a, int a_dtype, const double* b, int64_t n, double* d_part, double* d_out,
                       hipStream_t st) {
  hipLaunchKernelGGL(diff_norm_part, dim3(kNormBlocks), dim3(256), 0, st, a, a_dtype, b, n, d_part);
  hipLaunchKernelGGL(diff_norm_final, dim3(1), dim3(64), 0, st, d_part, kNormBlocks, d_out);
}

// ---------------------------------------------------------------- allocation-free form
// The partial sums of the norms in a static device array, for callers that cannot
// allocate.  Its size does not depend on n: every one of the kNormBlocks workgroups
// writes its two partials before the final kernel reads them (nothing has to start
// at zero).  Each device holds its own copy; calls that overlap on one device (other
// streams, other threads) share it and race.
namespace {
constexpr int kStaticNormElems = 2 * kNormBlocks;
__device__ __align__(256) double scratch[kStaticNormElems];

// Device address of `scratch` on each device, looked up once per device with that
// device current (host code must not use the symbol itself as a device pointer).
double* static_norm_scratch() {
  static std::mutex mu;
  static double* addr[64] = {};
  int dev = 0;
  TTNN_HIP(hipGetDevice(&dev));
  TTNN_REQUIRE(dev >= 0 && dev < 64, TTNN_E_INVALID, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    TTNN_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    TTNN_REQUIRE(p != nullptr, TTNN_E_HIP, "no device address for the static scratch");
    addr[dev] = static_cast<double*>(p);
  }
  return addr[dev];
}
}  // namespace

void launch_diff_norms_static(const void* a, int a_dtype, const double* b, int64_t n, double* d_out,
                              hipStream_t st) {
  static_assert(kStaticNormElems >= 2 * kNormBlocks, "the static scratch holds every partial");
  double* part = static_norm_scratch();
  launch_diff_norms(a, a_dtype, b, n, part, d_out, st);
}

}  // namespace ttnn
