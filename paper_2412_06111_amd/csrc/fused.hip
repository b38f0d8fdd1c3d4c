// Fused one-pass STTNN sketch for trees whose first root child A covers modes
// (1, 2) with two one-mode leaf children (e.g. ((1,2),(3,4)) and ((1,2),(3,(4,5)))).
//
// With M = T^{A} (n_A x n_B, n_A = n_1 n_2, column-major), the nodes A, {1}, {2}
// have S = {}, {}, {{1}} (Sec. 5, Fig. 5), so one pass over M produces
//   R_A = M X_A                                   (Sec. 5: A is sketched on T itself)
//   Z_A = Y_A^T M       -- the contraction T x_A Y_A^T reused by every node right of A
//   R_1 = T^{1} X_1     -- sum over columns of (n_1 x n_2 slab) . X_1 rows
//   R_2 = (T x_1 Y_1^T)^{2} X_2  -- Z1 = Y_1^T slab kept on chip, then Z1 . X_2 rows
// R_B and the right subtree (and the root sketch) follow from Z_A on the generic path.
//
// TTNN mode (template flag TT): R_A, Z_A and R_1 are the same sketches in TTNN (their
// reuse sets are empty), and for a root with two children R_B = T^{(B)} X_B with X_B
// rows over i_A, so R_B^T = X_B^T M is formed like Z_A, by the waves that STTNN spends
// on Z1.  The leaves right of A ({2} and the subtree of B) follow on the other paths.
//
// Each workgroup streams a tile of M (B2 slabs, one i2 and all of i1 each, by a range
// of columns) through LDS once; every product is an MFMA chain on that LDS tile:
//   (a)+(c) share the A fragments of the slab (rows i1, K = columns) against
//           [X_A | X_1] rows;  (b)+(d1) share its B fragments (K = i1) against
//           [Y_A | Y_1] rows;  (d2) contracts the LDS-staged Z1 over (j1, column)
//           (r = 16), or Z1 is written out for a streaming R_2 (r >= 32).
// Partial sums are written per tile in the accumulation precision and summed in a
// fixed order into the FP64 accumulators by sttnn_t4_reduce.
#include "fused.hpp"

#include <type_traits>

#include "engine.hpp"
#include "kernels.hpp"
#include "mfma.hpp"

namespace ttnn {
namespace {

constexpr int N1 = 128;

struct SttnnArgs {
  const void* T;
  int64_t n2, nA, nB;
  int TA, TB, CB;
  const void *XA, *X1, *YA, *Y1, *X2, *XB;
  void *PRA, *PZA, *PR1, *PR2, *PRB;
  void* Z1;            // Z1-out mode: Y_1^T slab for every (i_2, column), [i_2][i_B][j1]
};

// Wide fragment: V = 16 / sizeof(T) consecutive contraction values of one lane (one
// 16-byte load).  A 16 x 16 MFMA step takes KPL of them per lane group (BF16: all 8;
// FP32 / FP64: one), so a wide load feeds SUB = V / KPL MFMAs; sub-step s of every
// operand uses value s, and the SUB steps together cover the 4 V contraction values
// of the lane groups.  Every operand is laid out with the contraction index
// contiguous, in global memory and in LDS.
template <typename P>
struct Wide {
  using T = typename P::T;
  static constexpr int V = 16 / P::ESZ;
  static constexpr int SUB = V / P::KPL;
  static constexpr int KG = 4 * V;            // contraction values per wide step
  typedef T vec __attribute__((ext_vector_type(V)));
  __device__ static inline vec load(const T* p) { return *reinterpret_cast<const vec*>(p); }
  __device__ static inline typename P::Frag frag(const vec& w, int s) {
    if constexpr (P::KPL == 8) {
      (void)s;
      return __builtin_bit_cast(typename P::Frag, w);
    } else {
      return w[s];
    }
  }
};

// LDS plan of the kernel: the slab of T and the DRM rows of one sub-tile are copied
// straight from global memory into one of two LDS stages (global_load_lds, 16 bytes
// per lane, 64 lanes = whole rows per instruction) while the other stage is being
// consumed.  Operands that do not fit the budget are read from global memory (L2)
// instead.  Staged rows are not padded: the 16-byte chunks of row r are stored in
// XOR-swizzled order (chunk c at position c ^ (r mod 16, or mod the chunk count)),
// so reads along a row and gathers down a column spread over the LDS banks.
template <int DT, int R, int KP, int B2, int SC, bool TT, bool YR = false, bool ZO = false>
struct SttnnLayout {
  using P = Pol<DT>;
  using T = typename P::T;
  static constexpr int ESZ = P::ESZ;
  static constexpr int S = N1;                                // slab column stride
  static constexpr int SY = N1;                               // row stride of staged Y_A / Y_1 / X_B rows
  static constexpr int SXB = SY;
  static constexpr int SX = SC;                               // row stride of staged X_A / X_1 rows
  static constexpr size_t MS = size_t(SC) * S * ESZ;
  // Z1 stash rows (one per slab): FP32 rows are padded by 16 elements so that the four
  // rows read together by the 4 x 4 block products of (d2) fall on distinct banks
  static constexpr int ZPAD = DT == TTNN_F32 ? 16 : 0;
  static constexpr int ZS = KP * SC + ZPAD;
  // STTNN keeps Z1 = Y_1^T slab at FP32 accuracy whatever the plan dtype (the chained
  // intermediate of the sequential variant): a BF16 plan stashes FP32 values where Z1
  // is written out (ZF), and a high and a low BF16 half (hi = RNE(z), lo = RNE(z - hi),
  // |z - hi - lo| <= 2^-18 |z|) where it contracts Z1 with X_2 in the tile (ZH), so
  // that the BF16 MFMA takes both halves.
  static constexpr bool ZF = DT == TTNN_BF16 && ZO && !TT;
  static constexpr bool ZH = DT == TTNN_BF16 && !ZO && !TT;
  static constexpr int ZESZ = ZF ? 4 : ESZ;
  static constexpr size_t Z1 = TT ? 0 : size_t(ZH ? 2 : 1) * B2 * ZS * ZESZ;
  static constexpr size_t YAB = size_t(KP) * SY * ESZ;
  static constexpr size_t YB = YAB + (TT ? size_t(R) * SXB * ESZ : 0);
  static constexpr size_t XB = size_t(R) * SX * ESZ;
  static constexpr size_t BUDGET = 156 * 1024;
  // YR: the Y_A rows (TTNN: and the X_B rows) of the tile's B2 slabs stay in LDS for
  // the whole tile (one copy per tile instead of one per sub-tile), after both stages
  static constexpr size_t YRB = YR ? size_t(B2) * YB : 0;
  static constexpr bool STAGE_YA = !YR && 2 * (MS + YB) + Z1 <= BUDGET;
  // X_A / X_1 rows are staged where the Y_A rows are (staged or resident), and in FP64,
  // whose Y_A rows never fit: there every wave would otherwise load the same X fragments
  // from L2 inside its product loop
  static constexpr bool STAGE_X = (STAGE_YA || YR || DT == TTNN_F64) &&
                                  2 * (MS + (STAGE_YA ? YB : 0) + 2 * XB) + Z1 + YRB <= BUDGET;
  static constexpr size_t STAGE = MS + (STAGE_YA ? YB : 0) + (STAGE_X ? 2 * XB : 0);   // one stage
  static constexpr size_t Y1B = size_t(KP) * SY * ESZ;
  static constexpr bool STAGE_Y1 = !TT && 2 * STAGE + Z1 + YRB + Y1B <= BUDGET;
  static constexpr size_t OFF_YA = MS;                         // offsets within a stage
  static constexpr size_t OFF_XB = OFF_YA + YAB;               // TT: X_B rows after Y_A rows
  static constexpr size_t OFF_XA = OFF_YA + (STAGE_YA ? YB : 0);
  static constexpr size_t OFF_X1 = OFF_XA + (STAGE_X ? XB : 0);
  static constexpr size_t OFF_Z1 = 2 * STAGE;                 // after both stages
  static constexpr size_t OFF_YR = OFF_Z1 + Z1;
  static constexpr size_t OFF_Y1 = OFF_YR + YRB;
  static constexpr size_t TOTAL = OFF_Y1 + (STAGE_Y1 ? Y1B : 0);
};

constexpr int kThreadsF = 512;

// One lane's 16 bytes from global memory straight into LDS (global_load_lds_dwordx4);
// the LDS address is the wave's base plus 16 bytes per lane.
__device__ inline void lds_dma16(const void* g, void* l) {
  __builtin_amdgcn_global_load_lds(g, l, 16, 0, 0);
}

// XOR swizzle of the 16-byte chunks of a staged row of RL elements: element k of
// row r lives at r*RL + swz_off<T, RL>(r, k).
template <typename T, int RL>
struct Swz {
  static constexpr int EV = 16 / sizeof(T);
  static constexpr int CPR = RL / EV;                 // chunks per row
  static constexpr int MASK = (CPR < 16 ? CPR : 16) - 1;
  static_assert(CPR >= 1 && CPR <= 64 && (CPR & (CPR - 1)) == 0, "chunks per row");
  __device__ static inline int off(int r, int k) { return r * RL + ((((k / EV) ^ (r & MASK))) * EV) + (k % EV); }
};

// Copy `rows` rows of RL elements (row r from g + r*gs) into LDS at l, swizzled:
// each instruction fills 64 / CPR whole rows (64 lanes x 16 bytes, one contiguous
// kilobyte of LDS); lane L fetches the chunk that belongs at its position.
// Instructions are dealt to the eight waves; the LDS address is wave-uniform.
template <typename T, int RL>
__device__ inline void lds_dma_rows(const T* g, int64_t gs, T* l, int rows, int wave, int lane) {
  using Z = Swz<T, RL>;
  constexpr int RPI = 64 / Z::CPR;                    // rows per instruction
  const int ninstr = rows / RPI;
  const int rl = lane / Z::CPR, p = lane % Z::CPR;
  for (int q = wave; q < ninstr; q += kThreadsF / 64) {
    const int r = q * RPI + rl;
    const int c = p ^ (r & Z::MASK);
    lds_dma16(g + r * gs + static_cast<int64_t>(c) * Z::EV, l + q * RPI * RL);
  }
}

// Issue the copies of the sub-tile (slab i2, columns col0 .. col0+SC-1) into one stage.
template <int DT, int R, int KP, int B2, int SC, bool TT, bool YR, bool ZO>
__device__ inline void sttnn_issue(const SttnnArgs& a, char* sb, int64_t i2, int64_t col0, int wave, int lane) {
  using P = Pol<DT>;
  using Lay = SttnnLayout<DT, R, KP, B2, SC, TT, YR, ZO>;
  using T = typename P::T;
  const int64_t nA = a.nA, nB = a.nB, n2 = a.n2;
  lds_dma_rows<T, N1>(static_cast<const T*>(a.T) + i2 * N1 + nA * col0, nA, reinterpret_cast<T*>(sb), SC, wave,
                      lane);
  if constexpr (Lay::STAGE_YA) {
    lds_dma_rows<T, N1>(static_cast<const T*>(a.YA) + i2 * N1, nA, reinterpret_cast<T*>(sb + Lay::OFF_YA), KP, wave,
                        lane);
    if constexpr (TT)
      lds_dma_rows<T, N1>(static_cast<const T*>(a.XB) + i2 * N1, nA, reinterpret_cast<T*>(sb + Lay::OFF_XB), R, wave,
                          lane);
  }
  if constexpr (Lay::STAGE_X) {
    lds_dma_rows<T, SC>(static_cast<const T*>(a.XA) + col0, nB, reinterpret_cast<T*>(sb + Lay::OFF_XA), R, wave,
                        lane);
    lds_dma_rows<T, SC>(static_cast<const T*>(a.X1) + i2 * nB + col0, n2 * nB, reinterpret_cast<T*>(sb + Lay::OFF_X1),
                        R, wave, lane);
  }
}

// Wait for every outstanding LDS read of the wave (s_waitcnt lgkmcnt(0)).  While a
// global-to-LDS copy is in flight the compiler's own waits before an LDS operand
// cover all reads issued so far, including prefetches; waiting here, before the next
// step's reads are issued, lets those reads run under the current step's products.
__device__ inline void lds_wait_all() { __builtin_amdgcn_s_waitcnt(0xC07F); }

// acc[rb] += A[rb rows, K = i1] . slab[i1, column iBl] over the whole slab (K = N1),
// A rows delivered by loadA(rb, kk) (wide fragment at contraction offset kk).  The
// operands of step kw + 1 are loaded before the MFMAs of step kw are issued, so the
// LDS latency of one step is hidden behind the products of the previous one.
template <typename P, int NB, typename LoadA>
__device__ inline void bd_chain(const typename P::T* Ms, int iBl, int lg, LoadA&& loadA,
                                typename P::CFrag (&acc)[NB]) {
  using W = Wide<P>;
  using vec = typename W::vec;
  using ZN = Swz<typename P::T, N1>;
  constexpr int V = W::V, SUB = W::SUB, KG = W::KG, NK = N1 / KG;
  static_assert(NK % 2 == 0, "steps in pairs");
  auto load = [&](int kw, vec& bw, vec (&ay)[NB]) {
    const int kk = kw * KG + V * lg;
    bw = W::load(&Ms[ZN::off(iBl, kk)]);
#pragma unroll
    for (int rb = 0; rb < NB; ++rb) ay[rb] = loadA(rb, kk);
  };
  auto mma = [&](const vec& bw, const vec (&ay)[NB]) {
#pragma unroll
    for (int sb = 0; sb < SUB; ++sb)
#pragma unroll
      for (int rb = 0; rb < NB; ++rb) acc[rb] = P::mfma(W::frag(ay[rb], sb), W::frag(bw, sb), acc[rb]);
  };
  {
    vec bw0, ay0[NB], bw1, ay1[NB];
    load(0, bw0, ay0);
#pragma unroll
    // each wait, its loads and the products that follow stay in this order
    for (int kw = 0; kw < NK; kw += 2) {
      lds_wait_all();
      load(kw + 1, bw1, ay1);
      __builtin_amdgcn_sched_barrier(0);
      mma(bw0, ay0);
      __builtin_amdgcn_sched_barrier(0);
      lds_wait_all();
      if (kw + 2 < NK) load(kw + 2, bw0, ay0);
      __builtin_amdgcn_sched_barrier(0);
      mma(bw1, ay1);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// ZO (STTNN only): instead of contracting Z1 with X_2 in the tile (which re-reads the
// X_2 rows of the column band in every row tile), write Z1 out; R_2 is then one
// streaming contraction that reads X_2 once (used for r >= 32).
template <int DT, int R, int KP, int B2, int SC, bool TT, bool ZO>
__global__ __launch_bounds__(kThreadsF) void sttnn_t4_kernel(SttnnArgs a) {
  using P = Pol<DT>;
  using W = Wide<P>;
  // FP32 / BF16 Z1-out and TTNN forms at r = 32, and the BF16 Z1-out form at r = 64 (two
  // slabs per tile, 32-column sub-tiles): the tile's Y_A rows (and X_B rows) stay resident
  static constexpr bool YR = ((ZO || TT) && DT != TTNN_F64 && R == 32) || (DT == TTNN_BF16 && ZO && !TT && R == 64);
  using Lay = SttnnLayout<DT, R, KP, B2, SC, TT, YR, ZO>;
  using T = typename P::T;
  using Acc = typename P::Acc;
  using CFrag = typename P::CFrag;
  using vec = typename W::vec;
  constexpr int V = W::V, SUB = W::SUB, KG = W::KG;
  constexpr int CBR = R / 16;               // 16-wide column blocks of an R-wide output
  constexpr int KB = KP / 16;               // 16-row blocks of KP
  constexpr int KBB = R / 16;               // TT: 16-row blocks of R_B^T
  constexpr int NCB = SC / 16;              // 16-wide column blocks of a sub-tile
  static_assert(NCB == 4 || NCB == 2, "sub-tile width");
  constexpr int KT = KP * SC;               // (d2) contraction length per column sub-block
  constexpr int KW = KT / 8;                // per wave
  static_assert(KW % KG == 0 && SC % KG == 0 && N1 % KG == 0, "wide steps");
  // FP32 R_2 stage on 4 x 4 blocks (R <= 32; wider R keeps the 16 x 16 tiles, whose
  // accumulators are 4x smaller)
  constexpr bool D2Q = DT == TTNN_F32 && R <= 32;
  static_assert(!D2Q || KW % 64 == 0, "4 x 4 block steps");
  static_assert(Lay::TOTAL <= 160 * 1024, "LDS budget");
  static_assert(8 * 16 * R * sizeof(Acc) <= Lay::TOTAL, "reduction scratch");
  // With 32-column sub-tiles the (b)/(d1) products occupy waves 0-3 only; then (a)/(c)
  // go to waves 4-7 (two 16-row blocks of i1 each), so that each SIMD runs one wave of
  // either phase side by side instead of one wave alone through (b)/(d1).  Not where
  // the doubled accumulators would crowd the register file: FP64 at r >= 32, r = 64,
  // and, at r = 32, the forms that keep R_2 or R_B accumulators as well.
  constexpr bool SPLIT =
      NCB == 2 && (ZO || YR || R <= 16) && 2 * (B2 + 1) * CBR * int(sizeof(CFrag) / 4) <= 80;
  constexpr int RB1 = SPLIT ? 2 : 1;        // 16-row blocks of i1 per wave in (a)/(c)
  // (b)/(d1) chains software-pipelined where the second register set fits
  constexpr bool PIPE = DT != TTNN_F64 && (R <= 16 || (R == 32 && (ZO || (TT && DT == TTNN_F32))));

  __shared__ __align__(16) char smem[Lay::TOTAL];
  using ZT = typename std::conditional<Lay::ZF, float, T>::type;   // Z1 stash element
  ZT* Z1s = reinterpret_cast<ZT*>(smem + Lay::OFF_Z1);
  T* Z1lo = reinterpret_cast<T*>(smem + Lay::OFF_Z1) + B2 * Lay::ZS;   // ZH: the low halves
  T* Y1s = reinterpret_cast<T*>(smem + Lay::OFF_Y1);

  const int tid = threadIdx.x, lane = tid & 63, l16 = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform

  // tile of this workgroup.  Workgroups are dealt to the eight XCDs round robin; each
  // XCD takes a range of slab groups across every column band when TA allows, so the
  // tiles that share an L2 run through the same slabs in step and fetch each Y_A row
  // once between them (X_A, the smaller operand, is then shared by fewer tiles).
  int tA, tB;
  {
    const int w = blockIdx.x;
    if (a.TA % 8 == 0) {
      const int x = w % 8, j = w / 8, gpx = a.TA / 8;
      tA = x * gpx + j % gpx;
      tB = j / gpx;
    } else if (a.TB % 8 == 0) {
      const int x = w % 8, j = w / 8, bpx = a.TB / 8;
      tB = x * bpx + j / a.TA;
      tA = j % a.TA;
    } else {
      tB = w / a.TA;
      tA = w % a.TA;
    }
  }
  const int64_t i2_0 = static_cast<int64_t>(tA) * B2;
  const int64_t c_tile = static_cast<int64_t>(tB) * a.CB * SC;
  const T* XA = static_cast<const T*>(a.XA);
  const T* X1 = static_cast<const T*>(a.X1);
  const T* YA = static_cast<const T*>(a.YA);
  const T* Y1 = static_cast<const T*>(a.Y1);
  const T* X2 = static_cast<const T*>(a.X2);
  const T* XB = static_cast<const T*>(a.XB);
  const int64_t nA = a.nA, nB = a.nB, n2 = a.n2;

  auto stage_base = [&](int buf) -> char* { return smem + buf * Lay::STAGE; };
  // issue the copies of sub-tile s into stage buf
  auto issue = [&](int s, int buf) {
    const int cb = s / B2, i2l = s % B2;
    sttnn_issue<DT, R, KP, B2, SC, TT, YR, ZO>(a, stage_base(buf), i2_0 + i2l,
                                               c_tile + static_cast<int64_t>(cb) * SC, wave, lane);
  };
  // Y_1 rows, resident for the whole kernel; YR: the Y_A rows of the tile's slabs
  if constexpr (Lay::STAGE_Y1) lds_dma_rows<T, N1>(Y1, N1, Y1s, KP, wave, lane);
  T* YRs = reinterpret_cast<T*>(smem + Lay::OFF_YR);
  constexpr int YRN = KP + (TT ? R : 0);      // resident rows per slab: Y_A, then X_B
  if constexpr (YR) {
#pragma unroll
    for (int i2l = 0; i2l < B2; ++i2l) {
      lds_dma_rows<T, N1>(YA + (i2_0 + i2l) * N1, nA, YRs + i2l * YRN * N1, KP, wave, lane);
      if constexpr (TT) lds_dma_rows<T, N1>(XB + (i2_0 + i2l) * N1, nA, YRs + (i2l * YRN + KP) * N1, R, wave, lane);
    }
  }
  using ZN = Swz<T, N1>;                    // staged rows of N1 elements (slab columns, Y rows)
  using ZX = Swz<T, SC>;                    // staged rows of SC elements (X_A, X_1 rows)

  CFrag rA[RB1][B2][CBR];
  CFrag r1[RB1][CBR];
  CFrag r2[CBR];
  // FP32 (d2): 16 blocks of 4 x 4 per column group (block = lane / 4, row i2l = register
  // index, column 4 g + lane % 4); summed over blocks and waves at the end of the tile
  f32x4_t r2q[D2Q ? R / 4 : 1];
  CFrag zA[KB];
  CFrag zB[TT ? KBB : 1];
  const CFrag zero = {};
#pragma unroll
  for (int h = 0; h < RB1; ++h)
#pragma unroll
    for (int c = 0; c < CBR; ++c) {
      r1[h][c] = zero;
#pragma unroll
      for (int i = 0; i < B2; ++i) rA[h][i][c] = zero;
    }
#pragma unroll
  for (int c = 0; c < CBR; ++c) r2[c] = zero;
#pragma unroll
  for (int g = 0; g < (D2Q ? R / 4 : 1); ++g) r2q[g] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  // roles in the (b)/(d1) phase: Z_A, or Z1 (STTNN) / R_B^T (TTNN), for one 16-column
  // block of the sub-tile
  const bool bd_active = wave < 2 * NCB;
  const int cblk = wave % NCB;
  const bool bd_zA = (wave / NCB) == 0;
  const int iBl = 16 * cblk + l16;         // column of the sub-tile in the (b)/(d1) phase
  const bool ac_active = !SPLIT || wave >= 2 * NCB;
  const int i1base = SPLIT ? 32 * (wave - 2 * NCB) : 16 * wave;   // first i1 row of (a)/(c)

  const int nsub = a.CB * B2;
  issue(0, 0);
  for (int cb = 0; cb < a.CB; ++cb) {
    const int64_t iBbase = c_tile + static_cast<int64_t>(cb) * SC;
#pragma unroll
    for (int rb = 0; rb < KB; ++rb) zA[rb] = zero;
    if constexpr (TT) {
#pragma unroll
      for (int rb = 0; rb < KBB; ++rb) zB[rb] = zero;
    }

#pragma unroll
    for (int i2l = 0; i2l < B2; ++i2l) {
      const int s = cb * B2 + i2l;
      const int64_t i2 = i2_0 + i2l;
      const int buf = s & 1;
      __builtin_amdgcn_s_waitcnt(0);      // this wave's copies of sub-tile s have landed
      __syncthreads();                    // ... everyone's; and stage buf^1 is free again
      if (s + 1 < nsub) issue(s + 1, buf ^ 1);
      const T* Ms = reinterpret_cast<const T*>(stage_base(buf));
      const T* YAs = YR ? YRs + i2l * YRN * N1 : reinterpret_cast<const T*>(stage_base(buf) + Lay::OFF_YA);
      const T* XBs = YR ? YRs + (i2l * YRN + KP) * N1 : reinterpret_cast<const T*>(stage_base(buf) + Lay::OFF_XB);
      const T* XAs = reinterpret_cast<const T*>(stage_base(buf) + Lay::OFF_XA);
      const T* X1s = reinterpret_cast<const T*>(stage_base(buf) + Lay::OFF_X1);

      // (a) R_A rows of this slab and (c) R_1: A = slab (rows i1, K = columns)
      if constexpr (!SPLIT) {
        const int i1 = 16 * wave + l16;
#pragma unroll
        for (int kw = 0; kw < SC / KG; ++kw) {
          const int kk = kw * KG + V * lg;
          vec aw;
#pragma unroll
          for (int e = 0; e < V; ++e) aw[e] = Ms[ZN::off(kk + e, i1)];
          vec bA[CBR], b1[CBR];
#pragma unroll
          for (int c = 0; c < CBR; ++c) {
            const int j = 16 * c + l16;
            if constexpr (Lay::STAGE_X) {
              bA[c] = W::load(XAs + ZX::off(j, kk));
              b1[c] = W::load(X1s + ZX::off(j, kk));
            } else {
              bA[c] = W::load(XA + static_cast<int64_t>(j) * nB + iBbase + kk);
              b1[c] = W::load(X1 + (static_cast<int64_t>(j) * n2 + i2) * nB + iBbase + kk);
            }
          }
#pragma unroll
          for (int sb = 0; sb < SUB; ++sb) {
            const auto af = W::frag(aw, sb);
#pragma unroll
            for (int c = 0; c < CBR; ++c) {
              rA[0][i2l][c] = P::mfma(af, W::frag(bA[c], sb), rA[0][i2l][c]);
              r1[0][c] = P::mfma(af, W::frag(b1[c], sb), r1[0][c]);
            }
          }
        }
      } else if (ac_active) {
#pragma unroll
      for (int kw = 0; kw < SC / KG; ++kw) {
        const int kk = kw * KG + V * lg;
        vec aw[RB1];
#pragma unroll
        for (int h = 0; h < RB1; ++h)
#pragma unroll
          for (int e = 0; e < V; ++e) aw[h][e] = Ms[ZN::off(kk + e, i1base + 16 * h + l16)];
        vec bA[CBR], b1[CBR];
#pragma unroll
        for (int c = 0; c < CBR; ++c) {
          const int j = 16 * c + l16;
          if constexpr (Lay::STAGE_X) {
            bA[c] = W::load(XAs + ZX::off(j, kk));
            b1[c] = W::load(X1s + ZX::off(j, kk));
          } else {
            bA[c] = W::load(XA + static_cast<int64_t>(j) * nB + iBbase + kk);
            b1[c] = W::load(X1 + (static_cast<int64_t>(j) * n2 + i2) * nB + iBbase + kk);
          }
        }
#pragma unroll
        for (int sb = 0; sb < SUB; ++sb)
#pragma unroll
          for (int h = 0; h < RB1; ++h) {
            const auto af = W::frag(aw[h], sb);
#pragma unroll
            for (int c = 0; c < CBR; ++c) {
              rA[h][i2l][c] = P::mfma(af, W::frag(bA[c], sb), rA[h][i2l][c]);
              r1[h][c] = P::mfma(af, W::frag(b1[c], sb), r1[h][c]);
            }
          }
      }
      }  // ac_active

      // (b) Z_A += Y_A^T slab; (b') TTNN: R_B^T += X_B^T slab; (d1) STTNN: Z1 = Y_1^T slab.
      // B = slab (K = i1, columns)
      // (d1) result: the Z1 rows of this slab go to the LDS stash
      auto stash_z1 = [&](const CFrag (&acc)[KB]) {
#pragma unroll
        for (int rb = 0; rb < KB; ++rb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int j1 = 16 * rb + P::crow(lane, v);
            const int at = i2l * Lay::ZS + iBl * KP + j1;
            if constexpr (Lay::ZF) {
              Z1s[at] = acc[rb][v];
            } else if constexpr (Lay::ZH) {
              const T hi = P::from_acc(acc[rb][v]);
              Z1s[at] = hi;
              Z1lo[at] = P::from_acc(acc[rb][v] - bf16_bits_to_f32(hi));
            } else {
              Z1s[at] = P::from_acc(acc[rb][v]);
            }
          }
      };
      if constexpr (PIPE) {
        if (bd_active && bd_zA) {
          bd_chain<P, KB>(Ms, iBl, lg, [&](int rb, int kk) -> vec {
            const int jr = 16 * rb + l16;
            if constexpr (Lay::STAGE_YA || YR) return W::load(YAs + ZN::off(jr, kk));
            else return W::load(YA + static_cast<int64_t>(jr) * nA + i2 * N1 + kk);
          }, zA);
        } else if (TT && bd_active) {
          bd_chain<P, (TT ? KBB : 1)>(Ms, iBl, lg, [&](int rb, int kk) -> vec {
            const int jr = 16 * rb + l16;
            if constexpr (Lay::STAGE_YA || YR) return W::load(XBs + ZN::off(jr, kk));
            else return W::load(XB + static_cast<int64_t>(jr) * nA + i2 * N1 + kk);
          }, zB);
        } else if (!TT && bd_active) {
          CFrag acc[KB];
#pragma unroll
          for (int rb = 0; rb < KB; ++rb) acc[rb] = zero;
          bd_chain<P, KB>(Ms, iBl, lg, [&](int rb, int kk) -> vec {
            const int jr = 16 * rb + l16;
            if constexpr (Lay::STAGE_Y1) return W::load(Y1s + ZN::off(jr, kk));
            else return W::load(Y1 + static_cast<int64_t>(jr) * N1 + kk);
          }, acc);
          stash_z1(acc);
        }
      } else if (bd_active && bd_zA) {
#pragma unroll 2
        for (int kw = 0; kw < N1 / KG; ++kw) {
          const int kk = kw * KG + V * lg;
          const vec bw = W::load(&Ms[ZN::off(iBl, kk)]);
          vec ay[KB];
#pragma unroll
          for (int rb = 0; rb < KB; ++rb) {
            const int jr = 16 * rb + l16;
            if constexpr (Lay::STAGE_YA || YR) ay[rb] = W::load(YAs + ZN::off(jr, kk));
            else ay[rb] = W::load(YA + static_cast<int64_t>(jr) * nA + i2 * N1 + kk);
          }
#pragma unroll
          for (int sb = 0; sb < SUB; ++sb)
#pragma unroll
            for (int rb = 0; rb < KB; ++rb) zA[rb] = P::mfma(W::frag(ay[rb], sb), W::frag(bw, sb), zA[rb]);
        }
      } else if (TT && bd_active) {
#pragma unroll 2
        for (int kw = 0; kw < N1 / KG; ++kw) {
          const int kk = kw * KG + V * lg;
          const vec bw = W::load(&Ms[ZN::off(iBl, kk)]);
          vec ax[KBB];
#pragma unroll
          for (int rb = 0; rb < KBB; ++rb) {
            const int jr = 16 * rb + l16;
            if constexpr (Lay::STAGE_YA || YR) ax[rb] = W::load(XBs + ZN::off(jr, kk));
            else ax[rb] = W::load(XB + static_cast<int64_t>(jr) * nA + i2 * N1 + kk);
          }
#pragma unroll
          for (int sb = 0; sb < SUB; ++sb)
#pragma unroll
            for (int rb = 0; rb < KBB; ++rb) zB[rb] = P::mfma(W::frag(ax[rb], sb), W::frag(bw, sb), zB[rb]);
        }
      } else if (!TT && bd_active) {
        CFrag acc[KB];
#pragma unroll
        for (int rb = 0; rb < KB; ++rb) acc[rb] = zero;
#pragma unroll 2
        for (int kw = 0; kw < N1 / KG; ++kw) {
          const int kk = kw * KG + V * lg;
          const vec bw = W::load(&Ms[ZN::off(iBl, kk)]);
          vec ay[KB];
#pragma unroll
          for (int rb = 0; rb < KB; ++rb) {
            const int jr = 16 * rb + l16;
            if constexpr (Lay::STAGE_Y1) ay[rb] = W::load(Y1s + ZN::off(jr, kk));
            else ay[rb] = W::load(Y1 + static_cast<int64_t>(jr) * N1 + kk);
          }
#pragma unroll
          for (int sb = 0; sb < SUB; ++sb)
#pragma unroll
            for (int rb = 0; rb < KB; ++rb) acc[rb] = P::mfma(W::frag(ay[rb], sb), W::frag(bw, sb), acc[rb]);
        }
        stash_z1(acc);
      }
    }  // i2l
    // Z_A partials of this tile's row range for the sub-block's columns (before (d2),
    // so that the stores overlap it and zA's registers are free)
    if (bd_active && bd_zA) {
      Acc* PZA = static_cast<Acc*>(a.PZA);
      const int64_t iB = iBbase + iBl;
#pragma unroll
      for (int rb = 0; rb < KB; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int jA = 16 * rb + P::crow(lane, v);
          PZA[(static_cast<int64_t>(tA) * KP + jA) * nB + iB] = zA[rb][v];
        }
    }
    if constexpr (ZO) {
      // the tile's Z1 rows for this column block: B2 runs of SC * KP contiguous values
      __syncthreads();
      typedef ZT zvec __attribute__((ext_vector_type(16 / sizeof(ZT))));
      constexpr int ZV = 16 / sizeof(ZT);
      constexpr int NZ = SC * KP / ZV;
      ZT* Z1g = static_cast<ZT*>(a.Z1);
      for (int e = tid; e < B2 * NZ; e += kThreadsF) {
        const int i2l = e / NZ, q = e % NZ;
        const zvec v = *reinterpret_cast<const zvec*>(&Z1s[i2l * Lay::ZS + q * ZV]);
        *reinterpret_cast<zvec*>(&Z1g[((i2_0 + i2l) * nB + iBbase) * KP + q * ZV]) = v;
      }
    } else if constexpr (!TT && D2Q) {
      __syncthreads();
      // (d2) R_2[i2 rows] += Z1 (rows i2l, K = (column, j1)) . X_2 rows (column, j1) on
      // the 16-block 4 x 4 x 1 MFMA: only B2 <= 4 rows are live, so 16 x 16 tiles would
      // idle three quarters of the unit.  Block q = lane / 4 takes its own contraction
      // values (4 consecutive per wide load), lane % 4 is the row i2l for A and the
      // column within a group of 4 for B; group g covers columns 4 g .. 4 g + 3.
      const int q = lane >> 2, iq = lane & 3;
#pragma unroll
      for (int kw = 0; kw < KW / 64; ++kw) {
        const int K = wave * KW + kw * 64 + 4 * q;
        f32x4_t az;
        if (iq < B2) az = *reinterpret_cast<const f32x4_t*>(&Z1s[iq * Lay::ZS + K]);
        else az = f32x4_t{0.f, 0.f, 0.f, 0.f};
        f32x4_t bx[R / 4];
#pragma unroll
        for (int g = 0; g < R / 4; ++g)
          bx[g] = *reinterpret_cast<const f32x4_t*>(X2 + (static_cast<int64_t>(4 * g + iq) * nB + iBbase) * KP + K);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int g = 0; g < R / 4; ++g) r2q[g] = __builtin_amdgcn_mfma_f32_4x4x1f32(az[s], bx[g][s], r2q[g], 0, 0, 0);
      }
    } else if constexpr (!TT) {
      __syncthreads();
      // (d2) R_2[i2 rows] += Z1 (rows i2l, K = (column, j1)) . X_2 rows (column, j1);
      // fully unrolled so that every X_2 load of the wave is in flight at once
#pragma unroll
      for (int kw = 0; kw < KW / KG; ++kw) {
        const int K = wave * KW + kw * KG + V * lg;
        vec azw, azl;
        if (l16 < B2) azw = W::load(reinterpret_cast<const T*>(&Z1s[l16 * Lay::ZS + K]));
        else azw = vec{};
        if constexpr (Lay::ZH) {
          if (l16 < B2) azl = W::load(&Z1lo[l16 * Lay::ZS + K]);
          else azl = vec{};
        }
        vec bx[CBR];
#pragma unroll
        for (int c = 0; c < CBR; ++c) {
          const int j = 16 * c + l16;
          bx[c] = W::load(X2 + (static_cast<int64_t>(j) * nB + iBbase) * KP + K);
        }
#pragma unroll
        for (int sb = 0; sb < SUB; ++sb)
#pragma unroll
          for (int c = 0; c < CBR; ++c) {
            r2[c] = P::mfma(W::frag(azw, sb), W::frag(bx[c], sb), r2[c]);
            if constexpr (Lay::ZH) r2[c] = P::mfma(W::frag(azl, sb), W::frag(bx[c], sb), r2[c]);
          }
      }
    }

    // TTNN R_B^T partials of this tile's row range for the sub-block's columns
    if constexpr (TT) {
      if (bd_active && !bd_zA) {
        Acc* PRB = static_cast<Acc*>(a.PRB);
        const int64_t iB = iBbase + iBl;
#pragma unroll
        for (int rb = 0; rb < KBB; ++rb)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int j = 16 * rb + P::crow(lane, v);
            PRB[(static_cast<int64_t>(tA) * R + j) * nB + iB] = zB[rb][v];
          }
      }
    }
  }  // cb

  // ---- partial results of the tile
  if (ac_active) {
    Acc* PRA = static_cast<Acc*>(a.PRA);
    Acc* PR1 = static_cast<Acc*>(a.PR1);
#pragma unroll
    for (int h = 0; h < RB1; ++h)
#pragma unroll
      for (int c = 0; c < CBR; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i1 = i1base + 16 * h + P::crow(lane, v);
          const int j = 16 * c + l16;
#pragma unroll
          for (int i2l = 0; i2l < B2; ++i2l) {
            const int64_t iA = (i2_0 + i2l) * N1 + i1;
            PRA[(static_cast<int64_t>(tB) * nA + iA) * R + j] = rA[h][i2l][c][v];
          }
          PR1[((static_cast<int64_t>(tA) * a.TB + tB) * N1 + i1) * R + j] = r1[h][c][v];
        }
  }
  if constexpr (TT || ZO) return;
  __syncthreads();
  Acc* red = reinterpret_cast<Acc*>(smem);          // 8 waves x 16 rows x R
  if constexpr (D2Q) {
    // sum the 16 blocks (lanes 4 q + jj, q = 0..15) by a fixed butterfly; lanes 0..3 of
    // each wave then hold rows i2l = v, columns 4 g + lane
#pragma unroll
    for (int g = 0; g < R / 4; ++g)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float x = r2q[g][v];
        x += __shfl_xor(x, 4);
        x += __shfl_xor(x, 8);
        x += __shfl_xor(x, 16);
        x += __shfl_xor(x, 32);
        if (lane < 4) red[(wave * 16 + v) * R + 4 * g + lane] = x;
      }
  } else {
#pragma unroll
    for (int c = 0; c < CBR; ++c)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[(wave * 16 + P::crow(lane, v)) * R + 16 * c + l16] = r2[c][v];
  }
  __syncthreads();
  {
    Acc* PR2 = static_cast<Acc*>(a.PR2);
    for (int e = tid; e < B2 * R; e += kThreadsF) {
      const int row = e / R, j = e % R;
      Acc s = 0;
#pragma unroll
      for (int w = 0; w < 8; ++w) s += red[(w * 16 + row) * R + j];
      PR2[(static_cast<int64_t>(tB) * n2 + i2_0 + row) * R + j] = s;
    }
  }
}

// sum_{t < n} p[t * stride] in FP64 with eight interleaved partial sums (t mod 8),
// combined in a fixed order: eight loads in flight per thread.
template <typename Acc>
__device__ inline double sum_strided(const Acc* p, int n, int64_t stride) {
  double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int t = 0;
  for (; t + 8 <= n; t += 8) {
    Acc v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = p[(t + u) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u] += static_cast<double>(v[u]);
  }
  for (int q = 0; t < n; ++t, ++q) s[q] += static_cast<double>(p[t * stride]);
  return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// Tile of the transposing reductions: 16 output-fast x 32 input-fast entries per
// 256-thread block, two per thread.
constexpr int kRTX = 16, kRTY = 32;

// O[x + ldo y] (+)= alpha * sum_t P[t * tstride + x * ldx + y] for the tile (x0, y0):
// the partials are read along y (their contiguous index) and, through an LDS
// transpose, the output is written along x (its contiguous index).
template <typename Acc>
__device__ inline void reduce_transpose_tile(const Acc* P, int nt, int64_t tstride, int64_t ldx, int64_t X, int64_t Y,
                                             int64_t x0, int64_t y0, double* O, int64_t ldo, double alpha, bool acc,
                                             double (*tile)[kRTX + 1]) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int u = 0; u < kRTX * kRTY / 256; ++u) {
    const int e = tid + 256 * u;
    const int xl = e / kRTY, yl = e % kRTY;
    const int64_t x = x0 + xl, y = y0 + yl;
    double v = 0.0;
    if (x < X && y < Y) v = sum_strided(P + x * ldx + y, nt, tstride);
    tile[yl][xl] = v;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kRTX * kRTY / 256; ++u) {
    const int e = tid + 256 * u;
    const int xl = e % kRTX, yl = e / kRTX;
    const int64_t x = x0 + xl, y = y0 + yl;
    if (x < X && y < Y) {
      double* o = O + x + ldo * y;
      *o = acc ? *o + alpha * tile[yl][xl] : tile[yl][xl];
    }
  }
}

// Sum the tile partials in a fixed order into the FP64 state.  Blocks [0, nbA) do R_A
// (PRA [tB][iA][R] -> RA[iA + nA j]) and [nbA, nbA + nbZ) Z_A (PZA [tA][jA][iB] ->
// ZA[jA + k iB]) tile by tile, [nbA + nbZ, + nb1) R_1 (16 lanes per entry), and the
// remaining blocks the last segment, entry by entry: R_2 (mode 0, STTNN; PR2
// [tB][n2][R]), R_B (mode 1, TTNN; PRB [tA][R][nB]) or nothing (mode 2, STTNN with Z1
// written out).
template <typename Acc>
__global__ __launch_bounds__(256) void sttnn_t4_reduce(const Acc* PRA, const Acc* PZA, const Acc* PR1, const Acc* PR2,
                                                       int TA, int TB, int64_t n2, int64_t nA, int64_t nB, int R,
                                                       int KP, int k, double alpha, double* RA, double* ZA, double* R1,
                                                       double* R2, int tt, int nbA, int nbZ, int nb1) {
  __shared__ double tile[kRTY][kRTX + 1];
  const int64_t b = blockIdx.x;
  if (b < nbA) {
    const int64_t ty = (R + kRTY - 1) / kRTY;
    reduce_transpose_tile(PRA, TB, nA * R, R, nA, R, (b / ty) * kRTX, (b % ty) * kRTY, RA, nA, alpha, true, tile);
    return;
  }
  if (b < nbA + nbZ) {
    const int64_t bz = b - nbA;
    const int64_t tx = (k + kRTX - 1) / kRTX;
    reduce_transpose_tile(PZA, TA, static_cast<int64_t>(KP) * nB, nB, k, nB, (bz % tx) * kRTX, (bz / tx) * kRTY, ZA,
                          k, 1.0, false, tile);
    return;
  }
  const int64_t nR1 = static_cast<int64_t>(N1) * R;
  if (b < nbA + nbZ + nb1) {
    // R_1: TA * TB partials per entry, 16 lanes per entry (lane g sums partials
    // t = g mod 16), the 16 sums combined by a fixed butterfly
    const int g = threadIdx.x & 15;
    const int64_t f = ((b - nbA - nbZ) * blockDim.x + threadIdx.x) >> 4;
    if (f >= nR1) return;                       // whole 16-lane groups leave together
    const int64_t i1 = f / R, j = f % R;
    const int nt = TA * TB;
    const int64_t st = static_cast<int64_t>(N1) * R;
    double x = g < nt ? sum_strided(PR1 + i1 * R + j + g * st, (nt - g + 15) / 16, 16 * st) : 0.0;
    x += __shfl_xor(x, 8);
    x += __shfl_xor(x, 4);
    x += __shfl_xor(x, 2);
    x += __shfl_xor(x, 1);
    if (g == 0) R1[i1 + N1 * j] += alpha * x;
    return;
  }
  const int64_t nR2 = tt == 1 ? nB * R : tt == 0 ? n2 * R : 0;
  const int64_t nb = gridDim.x - nbA - nbZ - nb1;
  for (int64_t f = (b - nbA - nbZ - nb1) * blockDim.x + threadIdx.x; f < nR2; f += nb * blockDim.x) {
    if (tt == 0) {
      const int64_t i2 = f / R, j = f % R;
      R2[i2 + n2 * j] += alpha * sum_strided(PR2 + i2 * R + j, TB, n2 * R);
    } else {
      const int64_t j = f / nB, c = f % nB;
      R2[c + nB * j] += alpha * sum_strided(PR2 + j * nB + c, TA, static_cast<int64_t>(R) * nB);
    }
  }
}

// out[i0 + d0 (i1 + d1 i2)] = (valid) ? round(src[i0 s0 + i1 s1 + i2 s2]) : 0,
// valid: the coordinate `cdim` is below `lim`.
template <typename TO>
__global__ void gather_copy(const double* src, TO* out, int64_t d0, int64_t d1, int64_t d2, int64_t s0, int64_t s1,
                            int64_t s2, int cdim, int64_t lim) {
  const int64_t total = d0 * d1 * d2;
  for (int64_t o = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; o < total;
       o += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t i0 = o % d0, t = o / d0, i1 = t % d1, i2 = t / d1;
    const int64_t c = cdim == 0 ? i0 : cdim == 1 ? i1 : i2;
    double v = 0.0;
    if (c < lim) v = src[i0 * s0 + i1 * s1 + i2 * s2];
    if constexpr (sizeof(TO) == 2) {
      const uint32_t b = __float_as_uint(static_cast<float>(v));
      out[o] = static_cast<uint16_t>((b + 0x7FFFu + ((b >> 16) & 1u)) >> 16);
    } else {
      out[o] = static_cast<TO>(v);
    }
  }
}

}  // namespace

void copy_layout(const double* src, void* out, int dt, int64_t d0, int64_t d1, int64_t d2, int64_t s0, int64_t s1,
                 int64_t s2, int cdim, int64_t lim, hipStream_t st) {
  const int64_t total = d0 * d1 * d2;
  const int blocks = static_cast<int>(std::min<int64_t>((total + 255) / 256, 16384));
  if (dt == TTNN_BF16)
    hipLaunchKernelGGL(gather_copy<uint16_t>, dim3(blocks), dim3(256), 0, st, src, static_cast<uint16_t*>(out), d0,
                       d1, d2, s0, s1, s2, cdim, lim);
  else if (dt == TTNN_F32)
    hipLaunchKernelGGL(gather_copy<float>, dim3(blocks), dim3(256), 0, st, src, static_cast<float*>(out), d0, d1, d2,
                       s0, s1, s2, cdim, lim);
  else
    hipLaunchKernelGGL(gather_copy<double>, dim3(blocks), dim3(256), 0, st, src, static_cast<double*>(out), d0, d1,
                       d2, s0, s1, s2, cdim, lim);
}

namespace {

struct Shape {
  int B2, SC;
};

// Tile shape per dtype: B2 slabs of i_2 per tile, SC columns per sub-tile (sized so
// that the slab, the DRM rows of a sub-tile and the Z1 stash fit the LDS budget).
// The FP32 Z1-out and TTNN forms at r = 32 take two slabs, so that their Y_A (and X_B)
// rows stay in LDS.
template <int DT, int R, bool TT, bool ZO = false>
constexpr int b2_of() {
  return DT == TTNN_BF16 ? (R >= 64 ? 2 : (ZO || TT) && R == 32 ? 4 : 8)
         : DT == TTNN_F32 ? (R >= 64 || ((ZO || TT) && R == 32) ? 2 : 4)
                          : (R >= 64 || TT ? 2 : 4);
}
// BF16 Z1-out at r = 64 takes 32-column sub-tiles: with them the FP32 Z1 stash, the
// resident Y_A rows of both slabs and staged X_A / X_1 rows fit the LDS (at 64 columns
// the Y_A rows were re-copied every sub-tile and X_A / X_1 read from L2).
template <int DT, int R = 32, bool ZO = false>
constexpr int sc_of() {
  return DT == TTNN_BF16 ? (ZO && R >= 64 ? 32 : 64) : 32;
}

Shape shape_for(int dt, int R, bool tt, bool zout) {
  if (dt == TTNN_BF16) return {R >= 64 ? 2 : (zout || tt) && R == 32 ? 4 : 8, zout && !tt && R >= 64 ? 32 : 64};
  if (dt == TTNN_F32) return {R >= 64 || ((zout || tt) && R == 32) ? 2 : 4, 32};
  return {R >= 64 || tt ? 2 : 4, 32};
}

template <int DT, int R, int KP>
void launch_sttnn(bool tt, bool zout, const SttnnArgs& a, hipStream_t st) {
  constexpr int SC = sc_of<DT>(), SCZ = sc_of<DT, R, true>();
  constexpr int B2T = b2_of<DT, R, true>(), B2S = b2_of<DT, R, false>(), B2Z = b2_of<DT, R, false, true>();
  const dim3 grid(a.TA * a.TB);
  if (tt) hipLaunchKernelGGL((sttnn_t4_kernel<DT, R, KP, B2T, SC, true, false>), grid, dim3(kThreadsF), 0, st, a);
  else if (zout) hipLaunchKernelGGL((sttnn_t4_kernel<DT, R, KP, B2Z, SCZ, false, true>), grid, dim3(kThreadsF), 0, st, a);
  else hipLaunchKernelGGL((sttnn_t4_kernel<DT, R, KP, B2S, SC, false, false>), grid, dim3(kThreadsF), 0, st, a);
}

template <int DT>
void launch_sttnn_dt(int R, bool tt, bool zout, const SttnnArgs& a, hipStream_t st) {
  if (R == 16) launch_sttnn<DT, 16, 32>(tt, zout, a, st);
  else if (R == 32) launch_sttnn<DT, 32, 48>(tt, zout, a, st);
  else launch_sttnn<DT, 64, 96>(tt, zout, a, st);
}

int64_t elem_size(int dt) { return dt == TTNN_F64 ? 8 : dt == TTNN_F32 ? 4 : 2; }

}  // namespace

// ---------------------------------------------------------------- side stream
void fork_side(Plan& P, hipStream_t st, hipEvent_t after) {
  if (!P.side) {
    TTNN_HIP(hipStreamCreateWithFlags(&P.side, hipStreamNonBlocking));
    for (hipEvent_t& e : P.side_ev) TTNN_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  if (!after) {
    TTNN_HIP(hipEventRecord(P.side_ev[0], st));
    after = P.side_ev[0];
  }
  TTNN_HIP(hipStreamWaitEvent(P.side, after, 0));
}

void join_side(Plan& P, hipStream_t st) {
  if (!P.side_pending) return;
  TTNN_HIP(hipStreamWaitEvent(st, P.side_ev[1], 0));
  P.side_pending = false;
}

// ---------------------------------------------------------------- plan-time setup
void fused_prepare(Plan& P, hipStream_t st) {
  FusedT4& F = P.fused;
  F.enabled = false;
  const bool tt = P.variant == TTNN_TTNN;
  if (P.d < 3) return;
  const Node& root = P.nodes[0];
  if (root.children.size() < 2) return;
  if (tt && root.children.size() != 2) return;            // X_B rows must be exactly i_A
  const int A = root.children[0];
  const Node& nA_ = P.nodes[A];
  if (nA_.first != 0 || nA_.last != 1 || nA_.children.size() != 2) return;
  const int c1 = nA_.children[0], c2 = nA_.children[1];
  const Node &L1 = P.nodes[c1], &L2 = P.nodes[c2];
  if (!L1.leaf() || !L2.leaf()) return;
  const int R = nA_.r;
  if (L1.r != R || L2.r != R || L1.k != nA_.k || L2.k != nA_.k) return;
  int KP = 0;
  if (R == 16 && nA_.k <= 32) KP = 32;
  else if (R == 32 && nA_.k <= 48) KP = 48;
  else if (R == 64 && nA_.k <= 96) KP = 96;
  if (KP == 0) return;
  if (P.dims[0] != N1) return;
  const int64_t n2 = P.dims[1], nAs = N1 * n2, nB = P.N / nAs;
  // Z1-out form (STTNN, r >= 32): Z1 is written out and R_2 formed by one streaming
  // contraction that reads X_2 once, instead of re-reading X_2 in every row tile
  // (a BF16 plan writes Z1 in FP32 and contracts it with an FP32 copy of X_2)
  const int zdt = P.dtype == TTNN_BF16 ? TTNN_F32 : P.dtype;
  const bool zout = !tt && R >= 32 && right_mfma_eligible(static_cast<int64_t>(KP) * nB, n2, 1, R, zdt);
  const Shape sh = shape_for(P.dtype, R, tt, zout);
  if (n2 % sh.B2 != 0 || nB % sh.SC != 0) return;
  const int TA = static_cast<int>(n2 / sh.B2);
  // column tiles: the fewest that give every compute unit a tile (else as many as divide)
  int TB = 0;
  for (int cand = 1; cand <= 256; cand *= 2) {
    if (nB % (static_cast<int64_t>(sh.SC) * cand) != 0) continue;
    TB = cand;
    if (static_cast<int64_t>(TA) * cand >= 256) break;
  }
  if (TB == 0) return;
  F.R = R;
  F.KP = KP;
  F.k = nA_.k;
  F.B2 = sh.B2;
  F.SC = sh.SC;
  F.TA = TA;
  F.TB = TB;
  F.CB = static_cast<int>(nB / (static_cast<int64_t>(sh.SC) * TB));
  F.n2 = n2;
  F.nA = nAs;
  F.nB = nB;
  F.node_A = A;
  F.node_1 = c1;
  F.node_2 = c2;
  F.tt = tt;
  F.node_B = root.children[1];
  if (tt && (P.nodes[F.node_B].r != R || P.nodes[F.node_B].m != nAs)) return;

  const int dt = P.dtype;
  const int64_t es = elem_size(dt);
  // DRM copies in the fragment layouts of the kernel (the FP64 arrays of a lower-precision
  // plan hold the rounded values already, so these copies are exact)
  F.XA = P.alloc(es * nB * R);
  F.X1 = P.alloc(es * nAs / N1 * nB * R);
  F.YA = P.alloc(es * nAs * KP);
  const int x2dt = zout ? zdt : dt;
  if (tt) {
    F.XB = P.alloc(es * nAs * R);
  } else {
    F.Y1 = P.alloc(es * N1 * KP);
    F.X2 = P.alloc(elem_size(x2dt) * nB * KP * R);
  }
  const Node& NA = P.nodes[A];
  const double* XB64 = P.nodes[F.node_B].X64;
  const int k = nA_.k;
  // contraction index contiguous for every dtype
  if (!P.dry) {
    copy_layout(NA.X64, F.XA, dt, nB, R, 1, R, 1, 0, 0, nB, st);                     // [j][iB]
    copy_layout(L1.X64, F.X1, dt, nB, n2, R, n2 * R, R, 1, 0, nB, st);               // [j][i2][iB]
    copy_layout(NA.Y64, F.YA, dt, nAs, KP, 1, k, 1, 0, 1, k, st);                    // [jA][iA]
    if (tt) {
      copy_layout(XB64, F.XB, dt, nAs, R, 1, R, 1, 0, 1, R, st);                     // [j][iA]
    } else {
      copy_layout(L1.Y64, F.Y1, dt, N1, KP, 1, k, 1, 0, 1, k, st);                   // [j1][i1]
      copy_layout(L2.X64, F.X2, x2dt, KP, nB, R, R, static_cast<int64_t>(k) * R, 1, 0, k, st);  // [j][iB][j1]
    }
  }
  const int64_t as = dt == TTNN_F64 ? 8 : 4;
  F.PRA = P.alloc(as * TB * nAs * R);
  F.PZA = P.alloc(as * TA * KP * nB);
  F.PR1 = P.alloc(as * static_cast<int64_t>(TA) * TB * N1 * R);
  F.zout = zout;
  if (tt) F.PRB = P.alloc(as * TA * R * nB);
  else if (F.zout) F.Z1 = P.alloc(elem_size(zdt) * KP * n2 * nB);
  else F.PR2 = P.alloc(as * TB * n2 * R);
  F.enabled = true;
}

bool try_fused_update(Plan& P, const void* block, const int64_t* off, const int64_t* ext, double alpha,
                      hipStream_t st, std::vector<int>* done_nodes, std::vector<std::vector<int>>* done_prefixes) {
  const FusedT4& F = P.fused;
  if (!F.enabled) return false;
  for (int mu = 0; mu < P.d; ++mu)
    if (off[mu] != 0 || ext[mu] != P.dims[mu]) return false;
  SttnnArgs a;
  a.T = block;
  a.n2 = F.n2;
  a.nA = F.nA;
  a.nB = F.nB;
  a.TA = F.TA;
  a.TB = F.TB;
  a.CB = F.CB;
  a.XA = F.XA;
  a.X1 = F.X1;
  a.YA = F.YA;
  a.Y1 = F.Y1;
  a.X2 = F.X2;
  a.XB = F.XB;
  a.PRA = F.PRA;
  a.PZA = F.PZA;
  a.PR1 = F.PR1;
  a.PR2 = F.PR2;
  a.PRB = F.PRB;
  a.Z1 = F.Z1;
  if (P.dtype == TTNN_BF16) launch_sttnn_dt<TTNN_BF16>(F.R, F.tt, F.zout, a, st);
  else if (P.dtype == TTNN_F32) launch_sttnn_dt<TTNN_F32>(F.R, F.tt, F.zout, a, st);
  else launch_sttnn_dt<TTNN_F64>(F.R, F.tt, F.zout, a, st);
  if (P.timing) {
    TTNN_HIP(hipEventRecord(P.sweep_ev[1], st));
    P.sweep_recorded = true;
  }

  if (F.zout) {
    // R_2 += alpha Z1 X_2: Z1 [i_2][(i_B, j1)] against X_2 [j][(i_B, j1)], one pass over
    // both.  It needs only Z1 and X_2, so it runs on the plan's side stream beside the
    // partial reduction and the FP64 jobs that follow on the caller's stream (it uses the
    // partial scratch; the update joins it before any other user of that scratch).
    // Every kernel of this stretch streams from HBM or waits on it, so the overlap gains
    // little at FP32 (the kernels slow each other down); at BF16, where Z1 is half the
    // size, it does.
    fork_side(P, st, P.timing ? P.sweep_ev[1] : nullptr);   // the sweep's end event, when timed
    const int64_t K = static_cast<int64_t>(F.KP) * F.nB;
    const int zdt = P.dtype == TTNN_BF16 ? TTNN_F32 : P.dtype;      // Z1 and this X_2 copy
    const int nch = launch_right_mfma(F.Z1, zdt, K, F.n2, 1, F.X2, K, F.R, P.partial, P.partial_elems, P.side);
    const Node& n2d = P.nodes[F.node_2];
    launch_reduce(P.partial, nch, F.n2, F.R, 0, alpha, box_rows(P, n2d.first, n2d.last, off, ext), n2d.n, n2d.R, 1, 1,
                  P.side);
    TTNN_HIP(hipEventRecord(P.side_ev[1], P.side));
    P.side_pending = true;
  }

  const std::vector<int> pre{F.node_A};
  double* ZA = P.chain + P.prefix_offset.at(pre);
  const int node_last = F.tt ? F.node_B : F.node_2;
  const void* plast = F.tt ? F.PRB : F.PR2;
  const int64_t nbA = ((F.nA + kRTX - 1) / kRTX) * ((F.R + kRTY - 1) / kRTY);
  const int64_t nbZ = ((F.k + kRTX - 1) / kRTX) * ((F.nB + kRTY - 1) / kRTY);
  const int mode = F.tt ? 1 : F.zout ? 2 : 0;
  const int64_t nb1 = (static_cast<int64_t>(N1) * F.R * 16 + 255) / 256;
  const int64_t rest = (F.tt ? F.nB : F.zout ? 0 : F.n2) * F.R;
  const int64_t nbE = std::min<int64_t>((rest + 255) / 256, 2048);
  const dim3 grid(static_cast<unsigned>(nbA + nbZ + nb1 + nbE));
  if (P.dtype == TTNN_F64)
    hipLaunchKernelGGL(sttnn_t4_reduce<double>, grid, dim3(256), 0, st, static_cast<const double*>(F.PRA),
                       static_cast<const double*>(F.PZA), static_cast<const double*>(F.PR1),
                       static_cast<const double*>(plast), F.TA, F.TB, F.n2, F.nA, F.nB, F.R, F.KP, F.k, alpha,
                       P.nodes[F.node_A].R, ZA, P.nodes[F.node_1].R, P.nodes[node_last].R, mode,
                       static_cast<int>(nbA), static_cast<int>(nbZ), static_cast<int>(nb1));
  else
    hipLaunchKernelGGL(sttnn_t4_reduce<float>, grid, dim3(256), 0, st, static_cast<const float*>(F.PRA),
                       static_cast<const float*>(F.PZA), static_cast<const float*>(F.PR1),
                       static_cast<const float*>(plast), F.TA, F.TB, F.n2, F.nA, F.nB, F.R, F.KP, F.k, alpha,
                       P.nodes[F.node_A].R, ZA, P.nodes[F.node_1].R, P.nodes[node_last].R, mode,
                       static_cast<int>(nbA), static_cast<int>(nbZ), static_cast<int>(nb1));
  done_nodes->assign({F.node_A, F.node_1, node_last});
  done_prefixes->assign({pre});
  return true;
}

}  // namespace ttnn
