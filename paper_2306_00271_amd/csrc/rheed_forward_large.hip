// Forward propagation for 64 < N <= 128 beams on gfx950.
//
// The state Z = [c; c'] of a pair padded to 128 beams (two 128 x 128 complex
// blocks, 512 KB) does not fit on one CU, so it lives in a slot of device
// memory owned by the workgroup running the pair.  The RK stages act on the
// columns of Z independently (Sec. 3.4: the right-hand side is B(z) Z), so a
// slice is stepped in eight blocks of 16 columns: each wave of the 8-wave
// workgroup reads its 16 x 16 tile of the block's c and c' into registers,
// the s stages run with the stage input X_r of the block in LDS, and the tile
// goes back to memory.  Per slice the slot sees 1 MB of reads and writes
// against 7 x 8 x 128^3 flop (RK6), so the stage loop stays on the matrix
// cores.  The stages are the same Nystrom form as in the N <= 64 kernels:
// products G_r = M(z_i + c_r h) X_r with M = U + Gamma^2,
//   X_r = c + h c_r c' - h^2 sum_m (A^2)_{rm} G_m,
//   c <- c + h c' - h^2 sum_m (bA)_m G_m,   c' <- c' - h sum_m b_m G_m,
// each a complex 128 x 16 x 128 product in the 3-real-product form on
// v_mfma_f64_16x16x4f64, with U_{jk} = u_{g_j - g_k} gathered from the node's
// rod-difference table in LDS.
//
// After every slice the Gershgorin / Varah estimate of cond(Q), Q = c, over
// rows and columns < N decides the right-hand-side transformation
// Z <- Z Q^{-1} (Sec. 3.2, Algorithm 1).  It runs in two passes over rows held
// in registers (wave w: rows w + 8 m, two columns per lane): a column
// Gauss-Jordan elimination of Q with partial pivoting records the multipliers
// and pivot column of every step, Q E = Pi (E the product of the column
// operations, Pi a permutation); the same operations are then replayed on the
// rows of P, and P E with its columns put back in pivot order is P Q^{-1};
// c <- I.  The reflection (Eq. vrhocomp) eliminates Gamma Q - iP the same
// way; its first inverse column is E e_{pc_0}, formed by applying the recorded
// operations to a unit vector in reverse order, and rho = (Gamma Q + iP) x.
//
// The launch is a persistent grid of one workgroup per CU (the LDS holds one)
// over a cost-ordered pair list; no workgroup waits for another.
#include "rheed_large.h"
#include "rheed_gj.h"

namespace rheed {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int LW = 8;              // waves per workgroup
constexpr int LT = LW * 64;        // threads per workgroup
constexpr int LCB = 16;            // columns per block
constexpr int NCB = NL / LCB;      // column blocks
constexpr int LNE = 4;             // tile elements per lane (one 16 x 16 tile)
constexpr int LQ = NL / 4;         // k-steps of 4 in one product
constexpr int LRM = NL / LW;       // rows per wave in the eliminations

// Explicit RK tableaux in the Nystrom form above: node fraction c_r, the
// node's offset in the slice's table ring, A^2, bA and b (classical RK4 and
// Butcher's seventh-stage sixth-order method).
template <int S>
struct LTab;
template <>
struct LTab<0> {
  static constexpr int stages = 4, nodes = 2;
  static constexpr __device__ double c(int r) { return r == 0 ? 0.0 : r == 3 ? 1.0 : 0.5; }
  static constexpr __device__ int node(int r) { return r == 0 ? 0 : r == 3 ? 2 : 1; }
  static constexpr __device__ double a2(int r, int m) {
    return (r == 2 && m == 0) ? 0.25 : (r == 3 && m == 1) ? 0.5 : 0.0;
  }
  static constexpr __device__ double ba(int m) { return m < 3 ? 1.0 / 6.0 : 0.0; }
  static constexpr __device__ double b(int m) { return (m == 0 || m == 3) ? 1.0 / 6.0 : 1.0 / 3.0; }
};
template <>
struct LTab<1> {
  static constexpr int stages = 7, nodes = 4;
  static constexpr __device__ double c(int r) {
    return r == 0 ? 0.0 : r == 1 ? 1.0 / 3.0 : r == 2 ? 2.0 / 3.0 : r == 3 ? 1.0 / 3.0 : r == 6 ? 1.0 : 0.5;
  }
  static constexpr __device__ int node(int r) {  // c = 0, 1/3, 1/2, 2/3 -> 0..3; c = 1 -> 4
    return r == 0 ? 0 : r == 1 ? 1 : r == 2 ? 3 : r == 3 ? 1 : r == 6 ? 4 : 2;
  }
  static constexpr __device__ double a2(int r, int m) {
    return r == 2 ? (m == 0 ? 2.0 / 9.0 : 0.0)
         : r == 3 ? (m == 0 ? 1.0 / 9.0 : m == 1 ? -1.0 / 18.0 : 0.0)
         : r == 4 ? (m == 0 ? 11.0 / 32.0 : m == 1 ? -0.25 : m == 2 ? 1.0 / 32.0 : 0.0)
         : r == 5 ? (m == 0 ? 9.0 / 32.0 : m == 1 ? 1.0 / 16.0 : m == 2 ? -1.0 / 32.0 : m == 3 ? -3.0 / 16.0 : 0.0)
         : r == 6 ? (m == 0 ? -3.0 / 22.0 : m == 1 ? -3.0 / 22.0 : m == 2 ? 9.0 / 22.0 : m == 3 ? 12.0 / 11.0
                   : m == 4 ? -8.0 / 11.0 : 0.0)
         : 0.0;
  }
  static constexpr __device__ double ba(int m) {
    return m == 0 ? 11.0 / 120.0 : m == 2 ? 9.0 / 40.0 : m == 3 ? 9.0 / 20.0 : (m == 4 || m == 5) ? -2.0 / 15.0 : 0.0;
  }
  static constexpr __device__ double b(int m) {
    return (m == 0 || m == 6) ? 11.0 / 120.0 : (m == 2 || m == 3) ? 27.0 / 40.0 : (m == 4 || m == 5) ? -4.0 / 15.0 : 0.0;
  }
};

// The splitting stepper (BAB, Sec. 3.4): three kick positions per slice
// (0, g1, g1 + g2 of the slice) and the next slice's 0; weights come with the
// launch.
template <>
struct LTab<2> {
  static constexpr int stages = 3, nodes = 3;
};

struct LLds {
  double2 xb[NL * LCB];            // stage input of one column block; pivot rows during eliminations
  double2 tb[5][MAXBOXL + 1];      // node tables of the slice (ring); entry `box` of every row stays 0
  int bhk[NL][2];
  double g2s[NL];                  // Gamma_j^2, 0 on padding
  double rdg[NL], rof[NL];         // per row: |q_ii| and sum_{j != i} |q_ij| over j < N
  int pcrec[NL];                   // pivot column of every elimination step
  int pos[NL];                     // pivot step of every column in the last elimination
  unsigned gix[LQ / 2][LT];        // per thread: packed table indices of its A operand entries
  double2 xv[NL];                  // first column of the inverse in the reflection
  unsigned long long bnorm_bits;   // ||Gamma Q - iP||_inf and ||x||_inf of the reflection (bit patterns of
  unsigned long long xnorm_bits;   //   non-negative doubles, so an integer maximum orders them)
  int flag_singular;
  int bad;
};

// The LDS of the large kernel, in the forward kernels' shared allocation
// (rheed_forward_all.hip).
__device__ LLds& large_lds_ref();

struct LMat {
  double r[LNE];
  double i[LNE];
};

// Slot accesses name the global address space explicitly: through the
// pointers the out-of-line phases receive they would be flat instructions,
// which also count against the LDS counter, so every wait for an LDS read or
// a barrier would wait for the slot traffic as well.
typedef __attribute__((address_space(1))) double gdbl;
__device__ __forceinline__ double2 gld(const double2* p) {
  const gdbl* q = (const gdbl*)p;
  return make_double2(q[0], q[1]);
}
__device__ __forceinline__ void gst(double2* p, double2 v) {
  gdbl* q = (gdbl*)p;
  q[0] = v.x;
  q[1] = v.y;
}

// Rows m0 .. LRM-1 of z: column j <- column j - f_j column pc, with pc =
// 64 HF + pl (the pivot column's half is wave-uniform, so it selects code
// instead of data).
// Rows >= n (padding: unit rows of Q, zero rows of P and of the reflection
// matrix) have zeros in every pivot column and come out unchanged; the
// elimination skips them (m < m1, wave-uniform), the replay does not (there
// the per-row branch costs more registers than it saves).
template <int HF, int R>
__device__ __forceinline__ void col_update(double2 (&z)[R][2], int m0, int m1, int pl, double2 f0, double2 f1) {
#pragma unroll
  for (int m = 0; m < R; ++m) {
    if (m >= m0 && m < m1) {
      const double2 zp = make_double2(readlane_f64(z[m][HF].x, pl), readlane_f64(z[m][HF].y, pl));
      z[m][0].x = fma(-f0.x, zp.x, z[m][0].x);
      z[m][0].x = fma(f0.y, zp.y, z[m][0].x);
      z[m][0].y = fma(-f0.x, zp.y, z[m][0].y);
      z[m][0].y = fma(-f0.y, zp.x, z[m][0].y);
      z[m][1].x = fma(-f1.x, zp.x, z[m][1].x);
      z[m][1].x = fma(f1.y, zp.y, z[m][1].x);
      z[m][1].y = fma(-f1.x, zp.y, z[m][1].y);
      z[m][1].y = fma(-f1.y, zp.x, z[m][1].y);
    }
    // rows in groups of 4: the pivot-column reads of later rows are not
    // hoisted over earlier updates (their scalar copies would need registers)
    if ((m & 3) == 3) __builtin_amdgcn_sched_barrier(0);
  }
}

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// (U X) for the wave's 16 x 16 tile: A = U gathered from the node table,
// B = X of the block in LDS (row stride LCB).  Element v of the result
// belongs to row 16 w + 4 v + (lane >> 4), block column lane & 15.  F32:
// the same chains on v_mfma_f32_16x16x4f32 (the gather indices then hold
// the A rows in a_row<true> order), operands rounded to FP32, the chains
// combined in FP64.
template <int KQ, bool F32 = false>
__device__ __forceinline__ void gemm_tile(const double2* __restrict__ xb, const double2* __restrict__ tsl,
                                          const unsigned* __restrict__ gix, int lane, LMat& out) {
  __builtin_amdgcn_sched_barrier(0);
  using Acc = typename std::conditional<F32, f4, d4>::type;
  Acc t1 = Acc{0, 0, 0, 0}, t2 = t1, t3 = t1;
  int bb = (lane >> 4) * LCB + (lane & 15);
  asm volatile("" : "+v"(bb));  // keep the addresses from being hoisted out of the caller's loops
#pragma unroll
  for (int q = 0; q < KQ; ++q) {
    // packed gather indices from LDS (word q/2 of this thread), not held in registers
    const unsigned gw = gix[(q >> 1) * LT];
    const unsigned gi = (q & 1) ? (gw >> 16) : (gw & 0xffffu);
    const double2 u = tsl[gi];
    const double2 x = xb[bb + 4 * LCB * q];
    if constexpr (F32) {
      t1 = __builtin_amdgcn_mfma_f32_16x16x4f32((float)u.x, (float)x.x, t1, 0, 0, 0);
      t2 = __builtin_amdgcn_mfma_f32_16x16x4f32((float)u.y, (float)x.y, t2, 0, 0, 0);
      t3 = __builtin_amdgcn_mfma_f32_16x16x4f32((float)(u.x + u.y), (float)(x.x + x.y), t3, 0, 0, 0);
    } else {
      t1 = mfma(u.x, x.x, t1);
      t2 = mfma(u.y, x.y, t2);
      t3 = mfma(u.x + u.y, x.x + x.y, t3);
    }
    if ((q & 3) == 3) __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double a1 = t1[v], a2 = t2[v], a3 = t3[v];
    out.r[v] = a1 - a2;
    out.i[v] = a3 - a1 - a2;
  }
  __builtin_amdgcn_sched_barrier(0);
}

// One RK step of one column block: c, d (= c') of the wave's tile in, the
// stepped tile out.  xb holds X_r of the block while its product runs.
template <int STEPPER, int KQ>
__device__ __forceinline__ void step_block(LLds& s, LMat& c, LMat& d, const double (&g2)[4], int ob, int lane,
                                           int nb, double h) {
  using T = LTab<(STEPPER & 7)>;
  constexpr int SL = T::nodes + 1;
  const double hh = h * h;
  LMat G[T::stages];
  LMat cn, dn;
#pragma unroll
  for (int e = 0; e < LNE; ++e) {
    cn.r[e] = c.r[e] + h * d.r[e];
    cn.i[e] = c.i[e] + h * d.i[e];
    dn.r[e] = d.r[e];
    dn.i[e] = d.i[e];
  }
#pragma unroll
  for (int r = 0; r < T::stages; ++r) {
    const double hc = h * T::c(r);
#pragma unroll
    for (int e = 0; e < LNE; ++e) {
      double xr = c.r[e] + hc * d.r[e], xi = c.i[e] + hc * d.i[e];
#pragma unroll
      for (int m = 0; m < r; ++m) {
        if (T::a2(r, m) != 0.0) {
          xr -= hh * T::a2(r, m) * G[m].r[e];
          xi -= hh * T::a2(r, m) * G[m].i[e];
        }
      }
      s.xb[ob + 4 * LCB * e] = make_double2(xr, xi);
    }
    __syncthreads();
    gemm_tile<KQ, (STEPPER & F32_STAGES) != 0>(s.xb, s.tb[(nb + T::node(r)) % SL], &s.gix[0][threadIdx.x], lane, G[r]);
#pragma unroll
    for (int e = 0; e < LNE; ++e) {
      const double2 x = s.xb[ob + 4 * LCB * e];  // X_r back from LDS rather than kept in registers
      G[r].r[e] += g2[e] * x.x;
      G[r].i[e] += g2[e] * x.y;
      if (T::ba(r) != 0.0) {
        cn.r[e] -= hh * T::ba(r) * G[r].r[e];
        cn.i[e] -= hh * T::ba(r) * G[r].i[e];
      }
      dn.r[e] -= h * T::b(r) * G[r].r[e];
      dn.i[e] -= h * T::b(r) * G[r].i[e];
    }
    __syncthreads();
  }
  c = cn;
  d = dn;
}

// Column Gauss-Jordan elimination of the n x n leading block of the matrix
// whose rows w + 8 m sit in z[m] (column lane in [0], 64 + lane in [1]),
// recording what the other passes replay: the multipliers f of step k in
// frec[k][.] and its pivot column in pcrec[k].  Step k takes, among unused
// columns < n, the one with the largest |A_kj| (key: the upper 32 bits of
// |A_kj|^2 with the low 7 bits replaced by 127 - j, so near-ties go to the
// smaller index), pc; f_j = A_kj / A_k,pc and f_pc = 1 - 1 / A_k,pc; then
// column j <- column j - f_j column pc for every j, which leaves row k a unit
// row.  The columns already used are two wave-uniform bit masks (um0 for
// columns 0..63, um1 for 64..127), kept in scalar registers.  Rows of
// earlier blocks of 8 are unit rows with a zero in every later pivot column,
// so they are skipped.
template <int KB>
struct GjRec {
  static __device__ __forceinline__ void run(double2 (&z)[LRM][2], int n, int lane, int wu, unsigned long long& um0,
                                             unsigned long long& um1, double2* rowbuf, double2* frec, int* pcrec,
                                             int* flag_singular) {
    if (KB * LW >= n) return;
    const int mlim = (n - wu + LW - 1) / LW;  // this wave's rows < n
#pragma unroll 1
    for (int kk = 0; kk < LW; ++kk) {
      const int k = KB * LW + kk;
      if (k >= n) return;
      const int slot = k & 1;
      __syncthreads();
      const double2 v0 = rowbuf[slot * NL + lane], v1 = rowbuf[slot * NL + 64 + lane];
      const double m0 = v0.x * v0.x + v0.y * v0.y, m1 = v1.x * v1.x + v1.y * v1.y;
      unsigned k0 = 0, k1 = 0;
      if (!((um0 >> lane) & 1ull) && lane < n)
        k0 = ((unsigned)(((unsigned long long)__double_as_longlong(m0)) >> 32) & ~127u) | (unsigned)(127 - lane);
      if (!((um1 >> lane) & 1ull) && 64 + lane < n)
        k1 = ((unsigned)(((unsigned long long)__double_as_longlong(m1)) >> 32) & ~127u) | (unsigned)(63 - lane);
      const unsigned key = wave_max_u32(k0 > k1 ? k0 : k1);
      if ((key >> 7) == 0 && lane == 0 && wu == 0) *flag_singular = 1;
      const int pc = 127 - (int)(key & 127);
      const int hf = pc >> 6, pl = pc & 63;
      if (hf) um1 |= 1ull << pl;
      else um0 |= 1ull << pl;
      const double2 vs = hf ? v1 : v0;
      const double2 piv = make_double2(readlane_f64(vs.x, pl), readlane_f64(vs.y, pl));
      const double inv = 1.0 / (piv.x * piv.x + piv.y * piv.y);
      const double2 ip = make_double2(piv.x * inv, -piv.y * inv);
      double2 f0 = make_double2(v0.x * ip.x - v0.y * ip.y, v0.x * ip.y + v0.y * ip.x);
      double2 f1 = make_double2(v1.x * ip.x - v1.y * ip.y, v1.x * ip.y + v1.y * ip.x);
      if (lane == pl) {
        if (hf) f1 = make_double2(1.0 - ip.x, -ip.y);
        else f0 = make_double2(1.0 - ip.x, -ip.y);
      }
      if (wu == 0) {
        gst(&frec[k * NL + lane], f0);
        gst(&frec[k * NL + 64 + lane], f1);
        if (lane == 0) pcrec[k] = pc;
      }
      if (hf) col_update<1, LRM>(z, KB, mlim, pl, f0, f1);
      else col_update<0, LRM>(z, KB, mlim, pl, f0, f1);
      if (k + 1 < n && wu == (k + 1) % LW) {  // row k + 1: register KB, or KB + 1 after the block's last step
        constexpr int RB = KB + 1 < LRM ? KB + 1 : KB;
        const bool same = kk + 1 < LW;  // select values, not addresses, so z stays in registers
        const double2 a0 = z[KB][0], a1 = z[KB][1], b0 = z[RB][0], b1 = z[RB][1];
        rowbuf[(slot ^ 1) * NL + lane] = make_double2(same ? a0.x : b0.x, same ? a0.y : b0.y);
        rowbuf[(slot ^ 1) * NL + 64 + lane] = make_double2(same ? a1.x : b1.x, same ? a1.y : b1.y);
      }
    }
    GjRec<KB + 1>::run(z, n, lane, wu, um0, um1, rowbuf, frec, pcrec, flag_singular);
  }
};
template <>
struct GjRec<LRM> {
  static __device__ __forceinline__ void run(double2 (&)[LRM][2], int, int, int, unsigned long long&,
                                             unsigned long long&, double2*, double2*, int*, int*) {}
};

// Runs GjRec on the rows in z and leaves in s.pos the step at which each
// column was the pivot (its own index if never: columns >= n).
__device__ __forceinline__ void eliminate(double2 (&z)[LRM][2], int n, int lane, int w, LLds& s, double2* frec) {
  const int wu = __builtin_amdgcn_readfirstlane(w);
  unsigned long long um0 = 0, um1 = 0;
  double2* rowbuf = s.xb;
  __syncthreads();  // rowbuf aliases the stage buffer
  if (wu == 0) {
    rowbuf[lane] = z[0][0];
    rowbuf[64 + lane] = z[0][1];
  }
  GjRec<0>::run(z, n, lane, wu, um0, um1, rowbuf, frec, s.pcrec, &s.flag_singular);
  // the slot is read back by this workgroup only (one CU): workgroup-scope
  // ordering, which the barrier gives, is all it needs (a device-scope fence
  // would write back and invalidate the L2 that holds the multipliers)
  __syncthreads();
  const int tid = threadIdx.x;
  if (tid < NL) s.pos[tid] = tid;
  __syncthreads();
  if (tid < n) s.pos[s.pcrec[tid]] = tid;
  __syncthreads();
}

// z <- z E: the recorded column operations of steps 0 .. n-1 on R rows of
// this wave, rows w + 8 (m0 + m) for m < R (rows >= n are zero rows of P).
template <int R>
__device__ __forceinline__ void replay(double2 (&z)[R][2], int n, int lane, int w, int m0, const LLds& s,
                                       const double2* __restrict__ frec) {
  // two multiplier buffers, each loaded two steps before its use and used on
  // alternate steps: no register copies, so a step waits only for its own loads
  double2 a0 = gld(&frec[lane]), a1 = gld(&frec[64 + lane]);
  double2 b0 = a0, b1 = a1;
  if (n > 1) {
    b0 = gld(&frec[NL + lane]);
    b1 = gld(&frec[NL + 64 + lane]);
  }
#pragma unroll 1
  for (int k = 0; k < n; k += 2) {
    {
      const int pc = __builtin_amdgcn_readfirstlane(s.pcrec[k]);
      const int hf = pc >> 6, pl = pc & 63;
      if (hf) col_update<1, R>(z, 0, R, pl, a0, a1);
      else col_update<0, R>(z, 0, R, pl, a0, a1);
      if (k + 2 < n) {
        a0 = gld(&frec[(k + 2) * NL + lane]);
        a1 = gld(&frec[(k + 2) * NL + 64 + lane]);
      }
    }
    if (k + 1 < n) {
      const int pc = __builtin_amdgcn_readfirstlane(s.pcrec[k + 1]);
      const int hf = pc >> 6, pl = pc & 63;
      if (hf) col_update<1, R>(z, 0, R, pl, b0, b1);
      else col_update<0, R>(z, 0, R, pl, b0, b1);
      if (k + 3 < n) {
        b0 = gld(&frec[(k + 3) * NL + lane]);
        b1 = gld(&frec[(k + 3) * NL + 64 + lane]);
      }
    }
  }
  (void)w;
  (void)m0;
}

// Splitting step of one column block, tiles of c and c' from the slot and
// back: for r < nk, the kick c' <- c' - h w_r M(node n0 + r) c (the product
// on the matrix cores, c of the block as the B operand in LDS) and, with
// drift set, the drift c <- c + h a_r c'.
template <int KQ>
__device__ __forceinline__ void bab_block(double2* __restrict__ cg, double2* __restrict__ dg, int cb, int nk, int n0,
                                       double w0, double w1, double w2, double a0, double a1, double a2, bool drift,
                                       double h, int N) {
  LLds& s = large_lds_ref();
  constexpr int SL = LTab<2>::nodes + 1;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double g2[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) g2[v] = s.g2s[16 * w + 4 * v + (lane >> 4)];
  const int ob = (16 * w + (lane >> 4)) * LCB + (lane & 15);
  const int gb = (16 * w + (lane >> 4)) * NL + LCB * cb + (lane & 15);
  LMat c, d;
#pragma unroll
  for (int e = 0; e < LNE; ++e) {
    const double2 cv = gld(&cg[gb + 4 * NL * e]), dv = gld(&dg[gb + 4 * NL * e]);
    c.r[e] = cv.x;
    c.i[e] = cv.y;
    d.r[e] = dv.x;
    d.i[e] = dv.y;
  }
#pragma unroll 1
  for (int r = 0; r < nk; ++r) {
#pragma unroll
    for (int e = 0; e < LNE; ++e) s.xb[ob + 4 * LCB * e] = make_double2(c.r[e], c.i[e]);
    __syncthreads();
    LMat G;
    gemm_tile<KQ>(s.xb, s.tb[(n0 + r) % SL], &s.gix[0][tid], lane, G);
    const double hw = h * (r == 0 ? w0 : r == 1 ? w1 : w2);
#pragma unroll
    for (int e = 0; e < LNE; ++e) {
      d.r[e] -= hw * (G.r[e] + g2[e] * c.r[e]);
      d.i[e] -= hw * (G.i[e] + g2[e] * c.i[e]);
    }
    if (drift) {
      const double ha = h * (r == 0 ? a0 : r == 1 ? a1 : a2);
#pragma unroll
      for (int e = 0; e < LNE; ++e) {
        c.r[e] += ha * d.r[e];
        c.i[e] += ha * d.i[e];
      }
    }
    __syncthreads();
  }
  double pdg[4], pof[4];
#pragma unroll
  for (int e = 0; e < LNE; ++e) {
    gst(&cg[gb + 4 * NL * e], make_double2(c.r[e], c.i[e]));
    gst(&dg[gb + 4 * NL * e], make_double2(d.r[e], d.i[e]));
    const int row = 16 * w + 4 * e + (lane >> 4), col = LCB * cb + (lane & 15);
    const double av = sqrt(c.r[e] * c.r[e] + c.i[e] * c.i[e]);
    const bool in = row < N && col < N;
    pdg[e] = (in && row == col) ? av : 0.0;
    pof[e] = (in && row != col) ? av : 0.0;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      pdg[v] += __shfl_xor(pdg[v], off, 64);
      pof[v] += __shfl_xor(pof[v], off, 64);
    }
  }
  if ((lane & 15) == 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * w + 4 * v + (lane >> 4);
      s.rdg[row] = (cb == 0 ? 0.0 : s.rdg[row]) + pdg[v];
      s.rof[row] = (cb == 0 ? 0.0 : s.rof[row]) + pof[v];
    }
  }
}

// All column blocks of one splitting step, out of line: one call per slice,
// so the registers it saves and restores on entry and exit (to scratch, which
// reaches memory) are paid once per slice, not once per block.
template <int KQ>
__device__ __noinline__ void bab_all(double2* __restrict__ cg, double2* __restrict__ dg, int ncb, int nk, int n0,
                                     double w0, double w1, double w2, double a0, double a1, double a2, bool drift,
                                     double h, int N) {
#pragma unroll 1
  for (int cb = 0; cb < ncb; ++cb) bab_block<KQ>(cg, dg, cb, nk, n0, w0, w1, w2, a0, a1, a2, drift, h, N);
}

// The column blocks of a splitting step (blocks and k-steps stop at N as
// for the RK stages; the stepper runs every N <= 128, so down to one block).
__device__ __forceinline__ void bab_blocks(double2* cg, double2* dg, int ncb, int nk, int n0, double w0, double w1,
                                           double w2, const double (&a)[3], bool drift, double h, int N) {
#define RHEED_BAB(KQ)                                                                            \
  bab_all<KQ>(cg, dg, ncb, nk, n0, w0, w1, w2, a[0], a[1], a[2], drift, h, N);                    \
  break;
  switch (ncb) {
    case 1: RHEED_BAB(4)
    case 2: RHEED_BAB(8)
    case 3: RHEED_BAB(12)
    case 4: RHEED_BAB(16)
    case 5: RHEED_BAB(20)
    case 6: RHEED_BAB(24)
    case 7: RHEED_BAB(28)
    default: RHEED_BAB(32)
  }
#undef RHEED_BAB
}

template <int STEPPER, int KQ>
__device__ __forceinline__ void slice_block(double2* __restrict__ cg, double2* __restrict__ dg, int cb, int nb,
                                         double h, int N) {
  LLds& s = large_lds_ref();
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double g2[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) g2[v] = s.g2s[16 * w + 4 * v + (lane >> 4)];
  // the wave's tile: rows 16 w + 4 e + (lane >> 4), block column lane & 15
  const int ob = (16 * w + (lane >> 4)) * LCB + (lane & 15);
  const int gb = (16 * w + (lane >> 4)) * NL + LCB * cb + (lane & 15);
  LMat c, d;
#pragma unroll
  for (int e = 0; e < LNE; ++e) {
    const double2 cv = gld(&cg[gb + 4 * NL * e]), dv = gld(&dg[gb + 4 * NL * e]);
    c.r[e] = cv.x;
    c.i[e] = cv.y;
    d.r[e] = dv.x;
    d.i[e] = dv.y;
  }
  step_block<STEPPER, KQ>(s, c, d, g2, ob, lane, nb, h);
  double pdg[4], pof[4];
#pragma unroll
  for (int e = 0; e < LNE; ++e) {
    gst(&cg[gb + 4 * NL * e], make_double2(c.r[e], c.i[e]));
    gst(&dg[gb + 4 * NL * e], make_double2(d.r[e], d.i[e]));
    const int row = 16 * w + 4 * e + (lane >> 4), col = LCB * cb + (lane & 15);
    const double av = sqrt(c.r[e] * c.r[e] + c.i[e] * c.i[e]);
    const bool in = row < N && col < N;
    pdg[e] = (in && row == col) ? av : 0.0;
    pof[e] = (in && row != col) ? av : 0.0;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      pdg[v] += __shfl_xor(pdg[v], off, 64);
      pof[v] += __shfl_xor(pof[v], off, 64);
    }
  }
  if ((lane & 15) == 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * w + 4 * v + (lane >> 4);
      s.rdg[row] = (cb == 0 ? 0.0 : s.rdg[row]) + pdg[v];
      s.rof[row] = (cb == 0 ? 0.0 : s.rof[row]) + pof[v];
    }
  }
}

// All column blocks of one slice, out of line: one call per slice, so the
// registers it saves and restores on entry and exit (to scratch, which
// reaches memory) are paid once per slice, not once per block.
template <int STEPPER, int KQ>
__device__ __noinline__ void slice_all(double2* __restrict__ cg, double2* __restrict__ dg, int ncb, int nb, double h,
                                       int N) {
#pragma unroll 1
  for (int cb = 0; cb < ncb; ++cb) slice_block<STEPPER, KQ>(cg, dg, cb, nb, h, N);
}

// Recording elimination (see GjRec) of Q = c (which = 0) or of the
// reflection's Gamma Q - iP (which = 1), rows from the slot; the pivot step of
// every column goes to s.pos.  Out of line, with n and which made
// wave-uniform, so that its row predicates are scalar branches and its
// registers are allocated for this loop alone.
__device__ __noinline__ void elim_record(const double2* __restrict__ cg, const double2* __restrict__ dg,
                                         double2* __restrict__ frec, int N, int which) {
  LLds& s = large_lds_ref();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int n = __builtin_amdgcn_readfirstlane(N);
  double2 z[LRM][2];
  if (__builtin_amdgcn_readfirstlane(which) == 0) {
#pragma unroll
    for (int m = 0; m < LRM; ++m) {
      z[m][0] = gld(&cg[(w + LW * m) * NL + lane]);
      z[m][1] = gld(&cg[(w + LW * m) * NL + 64 + lane]);
    }
  } else {
#pragma unroll
    for (int m = 0; m < LRM; ++m) {
      const int row = w + LW * m;
      const double g2v = s.g2s[row];
      const double g_r = g2v >= 0.0 ? sqrt(g2v) : 0.0, g_i = g2v >= 0.0 ? 0.0 : -sqrt(-g2v);
#pragma unroll
      for (int hf = 0; hf < 2; ++hf) {
        const double2 cv = gld(&cg[row * NL + 64 * hf + lane]), pv = gld(&dg[row * NL + 64 * hf + lane]);
        z[m][hf] = make_double2(g_r * cv.x - g_i * cv.y + pv.y, g_r * cv.y + g_i * cv.x - pv.x);
      }
    }
  }
  eliminate(z, n, lane, w, s, frec);
}

// P <- P Q^{-1} after elim_record(which = 0): the recorded column operations
// replayed on the rows of P, each column put at its pivot step; c <- I.
__device__ __noinline__ void replay_p(double2* __restrict__ cg, double2* __restrict__ dg,
                                      const double2* __restrict__ frec, int N) {
  LLds& s = large_lds_ref();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int n = __builtin_amdgcn_readfirstlane(N);
  const int p0 = s.pos[lane], p1 = s.pos[64 + lane];
  // the rows of P are independent here: two passes of LRM / 2 rows per wave
  // keep the replay within the register budget
#pragma unroll 1
  for (int part = 0; part < 2; ++part) {
    constexpr int R = LRM / 2;
    const int m0 = part * R;
    double2 z[R][2];
#pragma unroll
    for (int m = 0; m < R; ++m) {
      z[m][0] = gld(&dg[(w + LW * (m0 + m)) * NL + lane]);
      z[m][1] = gld(&dg[(w + LW * (m0 + m)) * NL + 64 + lane]);
    }
    replay<R>(z, n, lane, w, m0, s, frec);
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int row = w + LW * (m0 + m);
      gst(&dg[row * NL + p0], z[m][0]);
      gst(&dg[row * NL + p1], z[m][1]);
      gst(&cg[row * NL + lane], make_double2(row == lane ? 1.0 : 0.0, 0.0));
      gst(&cg[row * NL + 64 + lane], make_double2(row == 64 + lane ? 1.0 : 0.0, 0.0));
    }
  }
  __syncthreads();
}

// Q^{-1} (or B^{-1} of the reflection) after elim_record: the recorded
// column operations replayed on the rows of I, each column put at its pivot
// step as in replay_p; written, all NL rows, to out (row major, stride NL).
__device__ __noinline__ void replay_identity(double2* __restrict__ out, const double2* __restrict__ frec, int N) {
  LLds& s = large_lds_ref();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int n = __builtin_amdgcn_readfirstlane(N);
  const int p0 = s.pos[lane], p1 = s.pos[64 + lane];
#pragma unroll 1
  for (int part = 0; part < 2; ++part) {
    constexpr int R = LRM / 2;
    const int m0 = part * R;
    double2 z[R][2];
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int row = w + LW * (m0 + m);
      z[m][0] = make_double2(row == lane ? 1.0 : 0.0, 0.0);
      z[m][1] = make_double2(row == 64 + lane ? 1.0 : 0.0, 0.0);
    }
    replay<R>(z, n, lane, w, m0, s, frec);
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int row = w + LW * (m0 + m);
      gst(&out[row * NL + p0], z[m][0]);
      gst(&out[row * NL + p1], z[m][1]);
    }
  }
}

// Copy of an NL x NL block of the slot (for the states the adjoint reads).
__device__ __forceinline__ void copy_block(double2* __restrict__ dst, const double2* __restrict__ src) {
  for (int e = threadIdx.x; e < NL * NL; e += LT) gst(&dst[e], gld(&src[e]));
}

// SAVE: keep the states the adjoint reads (a separate instance, so that the
// forward-only code keeps its own register allocation).
template <int STEPPER, bool SAVE>
__device__ void run_pair(const LargeArgs& A, int p, char* slot) {
  static_assert(!(SAVE && (STEPPER & F32_STAGES)), "FP32 stages run forward only");
  using T = LTab<(STEPPER & 7)>;
  constexpr int SL = T::nodes + 1;
  const FwdArgs& a = A.f;
  LLds& s = large_lds_ref();
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double2* __restrict__ cg = reinterpret_cast<double2*>(slot + LSLOT_C);
  double2* __restrict__ dg = reinterpret_cast<double2*>(slot + LSLOT_D);
  double2* __restrict__ frec = reinterpret_cast<double2*>(slot + LSLOT_F);
  const StructDev S = a.structs[a.pair_struct[p]];
  const int N = S.n_beams;
  const int L = S.n_slices;
  const double h = S.h;
  const double2* __restrict__ Us = a.U + S.table_off;
  const int ncb = (N + LCB - 1) / LCB;  // column blocks holding columns < N (5 .. 8; 1 .. 8 for splitting)
  // states kept for the adjoint (RK steppers): the state at the start of
  // every ck.every-th slice and after the last, T = Q^{-1} and (ck.every > 1)
  // R of every transformation, one decision byte per slice, and B^{-1} of
  // the reflection solve, all padded to NL
  constexpr bool save = SAVE && STEPPER != 2;
  char* pws = save ? a.ws + (long long)p * a.ck.pair_stride : nullptr;
  constexpr long long MATB = (long long)NL * NL * sizeof(double2);

  if (tid < NL) {
    s.bhk[tid][0] = tid < N ? a.beams[2 * (S.beam_off + tid)] : 0;
    s.bhk[tid][1] = tid < N ? a.beams[2 * (S.beam_off + tid) + 1] : 0;
  }
  if (tid == 0) {
    s.flag_singular = 0;
    s.bad = 0;
  }
  if (tid < SL) s.tb[tid][S.box] = make_double2(0.0, 0.0);
  __syncthreads();
  const double th0 = a.angles[2 * p], th1 = a.angles[2 * p + 1];
  if (tid < NL) {
    // Gamma_j^2 = gamma^2 - |b0 + k_j|^2 (Sec. 2.1), b0 = gamma cos(theta0) (cos theta1, sin theta1)
    const double b0x = S.gamma * cos(th0) * cos(th1);
    const double b0y = S.gamma * cos(th0) * sin(th1);
    double arg = 0.0;
    if (tid < N) {
      const double qx = b0x + s.bhk[tid][0] * S.recip[0] + s.bhk[tid][1] * S.recip[2];
      const double qy = b0y + s.bhk[tid][0] * S.recip[1] + s.bhk[tid][1] * S.recip[3];
      arg = S.gamma * S.gamma - (qx * qx + qy * qy);
    }
    s.g2s[tid] = arg;
  }
  __syncthreads();
  // gather indices of U_{ik} = u_{g_i - g_k} for the thread's A operand entries
  // (row 16 w + (lane & 15), k = 4 q + (lane >> 4)); padding reads entry `box` = 0
  {
    const int W = 2 * S.kd + 1;
    const int iA = 16 * w + a_row<(STEPPER & F32_STAGES) != 0>(lane & 15);
    const int baseA = (s.bhk[iA][0] + S.hd) * W + (s.bhk[iA][1] + S.kd);
#pragma unroll 4
    for (int q = 0; q < LQ; q += 2) {
      const int k0 = 4 * q + (lane >> 4), k1 = 4 * (q + 1) + (lane >> 4);
      const unsigned i0 = (iA < N && k0 < N) ? baseA - (s.bhk[k0][0] * W + s.bhk[k0][1]) : S.box;
      const unsigned i1 = (iA < N && k1 < N) ? baseA - (s.bhk[k1][0] * W + s.bhk[k1][1]) : S.box;
      s.gix[q >> 1][tid] = i0 | (i1 << 16);
    }
  }
  // Z0 = [I; i Gamma] (spans the columns of S^{-1}[I; O] of Algorithm 1), rows
  // of the state row major in the slot
  for (int e = tid; e < NL * NL; e += LT) {
    const int row = e / NL, col = e - row * NL;
    const double g2v = s.g2s[row];
    const bool dgn = row == col;
    gst(&cg[e], make_double2(dgn ? 1.0 : 0.0, 0.0));
    gst(&dg[e], make_double2((dgn && g2v < 0.0) ? sqrt(-g2v) : 0.0, (dgn && g2v >= 0.0) ? sqrt(g2v) : 0.0));
  }
  for (int e = tid; e < S.box; e += LT) s.tb[0][e] = Us[e];
  int nrhst = 0;

#pragma unroll 1
  for (int i = 0; i < L; ++i) {
    const int nb = i * T::nodes;
    {  // this slice's nodes after c = 0 (node nb came with the previous slice)
      const int total = T::nodes * S.box;
      for (int e = tid; e < total; e += LT) {
        const int q = e / S.box, j = e - q * S.box;
        s.tb[(nb + 1 + q) % SL][j] = Us[(long long)(nb + 1 + q) * S.box + j];
      }
    }
    __syncthreads();
    if (save && (i % a.ck.every) == 0) {
      double2* st = reinterpret_cast<double2*>(pws + (long long)(i / a.ck.every) * a.ck.state_bytes);
      copy_block(st, cg);
      copy_block(st + NL * NL, dg);
    }
    if constexpr (STEPPER == 2) {
      // kicks at the slice's nodes 0, g1, g1 + g2 with drifts between; the
      // slice's last kick (at its end, the next slice's 0) is merged into the
      // next slice's first: kicks act on c' from the left, so they commute
      // with the transformation (a right multiplication) and leave Q = c,
      // and with it the badness, as they are
      const double w0 = i == 0 ? A.sp_b[0] : A.sp_b[0] + A.sp_b[3];
      const double adr[3] = {A.sp_a[0], A.sp_a[1], A.sp_a[2]};
      bab_blocks(cg, dg, ncb, 3, nb, w0, A.sp_b[1], A.sp_b[2], adr, true, h, N);
    } else {
    // column blocks and k-steps past N hold zeros only (padding columns of
    // c and c' stay as they are, U_jk = 0 for k >= N), so both stop at N
    switch (ncb) {
      case 5:
        slice_all<STEPPER, 20>(cg, dg, 5, nb, h, N);
        break;
      case 6:
        slice_all<STEPPER, 24>(cg, dg, 6, nb, h, N);
        break;
      case 7:
        slice_all<STEPPER, 28>(cg, dg, 7, nb, h, N);
        break;
      default:
        slice_all<STEPPER, 32>(cg, dg, NCB, nb, h, N);
        break;
    }
    }
    __syncthreads();
    // condition estimate of Q = c (Sec. 3.2): the Gershgorin / Varah bound
    // max_i(|q_ii| + r_i) / min_i(|q_ii| - r_i), r_i = sum_{j != i} |q_ij|
    bool do_rhst;
    {
      double hi = 0.0, lo = 1.0e308;
#pragma unroll
      for (int hf = 0; hf < 2; ++hf) {
        const int row = 64 * hf + lane;
        if (row < N) {
          const double dv = s.rdg[row], ov = s.rof[row];
          hi = fmax(hi, dv + ov);
          lo = fmin(lo, dv - ov);
        }
      }
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        hi = fmax(hi, __shfl_xor(hi, off, 64));
        lo = fmin(lo, __shfl_xor(lo, off, 64));
      }
      const double xi = lo > 0.0 ? hi / lo : INFINITY;
      do_rhst = xi > a.threshold;
    }
    if (save && tid == 0) pws[a.ck.flags_off + i] = do_rhst ? 1 : 0;
    if (do_rhst) {
      // Z <- Z Q^{-1}: eliminate Q (recording), replay on the rows of P
      ++nrhst;
      elim_record(cg, dg, frec, N, 0);
      if (save) replay_identity(reinterpret_cast<double2*>(pws + a.ck.q_off + (long long)i * MATB), frec, N);
      replay_p(cg, dg, frec, N);
      if (save && a.ck.r_off) {  // R = P Q^{-1} for an adjoint that keeps states only every few slices
        copy_block(reinterpret_cast<double2*>(pws + a.ck.r_off + (long long)i * MATB), dg);
        __syncthreads();
      }
    }
  }

  if constexpr (STEPPER == 2) {  // the last slice's final kick, at z = 0
    const double adr[3] = {0.0, 0.0, 0.0};
    bab_blocks(cg, dg, ncb, 1, L * T::nodes, A.sp_b[3], 0.0, 0.0, adr, false, h, N);
    __syncthreads();
  }
  if (save) {  // the final state
    double2* st = reinterpret_cast<double2*>(pws + (long long)(a.ck.max_ckpt - 1) * a.ck.state_bytes);
    copy_block(st, cg);
    copy_block(st + NL * NL, dg);
  }
  // reflection (Eq. vrhocomp): upper = Gamma Q - iP, lower = Gamma Q + iP,
  // rho = lower x with upper x = e_1
  elim_record(cg, dg, frec, N, 1);
  if (save) replay_identity(reinterpret_cast<double2*>(pws + a.ck.binv_off), frec, N);
  if (w == 0) {
    // x = E e_{pc_0}: the recorded operations in reverse order, each
    // v <- v - e_pc (f . v)
    const int pc0 = s.pcrec[0];
    double2 v0 = make_double2(lane == pc0 ? 1.0 : 0.0, 0.0), v1 = make_double2(64 + lane == pc0 ? 1.0 : 0.0, 0.0);
#pragma unroll 1
    for (int k = N - 1; k >= 0; --k) {
      const double2 f0 = gld(&frec[k * NL + lane]), f1 = gld(&frec[k * NL + 64 + lane]);
      double sr = (f0.x * v0.x - f0.y * v0.y) + (f1.x * v1.x - f1.y * v1.y);
      double si = (f0.x * v0.y + f0.y * v0.x) + (f1.x * v1.y + f1.y * v1.x);
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        sr += __shfl_xor(sr, off, 64);
        si += __shfl_xor(si, off, 64);
      }
      const int pc = __builtin_amdgcn_readfirstlane(s.pcrec[k]);
      if (lane == (pc & 63)) {
        if (pc >> 6) v1 = make_double2(v1.x - sr, v1.y - si);
        else v0 = make_double2(v0.x - sr, v0.y - si);
      }
    }
    s.xv[lane] = v0;
    s.xv[64 + lane] = v1;
  }
  if (tid == 0) {
    s.bnorm_bits = 0;
    s.xnorm_bits = 0;
  }
  __syncthreads();
  if (tid < a.ld) {
    const int j = tid;
    double eta = 0.0;
    double2 rj = make_double2(0.0, 0.0);
    if (j < N) {
      const double g2v = s.g2s[j];
      const double g_r = g2v >= 0.0 ? sqrt(g2v) : 0.0, g_i = g2v >= 0.0 ? 0.0 : -sqrt(-g2v);
      double rs = 0.0;  // row j of Gamma Q - iP, for the breakdown test
      for (int k = 0; k < N; ++k) {
        const double2 cv = gld(&cg[j * NL + k]), pv = gld(&dg[j * NL + k]), x = s.xv[k];
        const double lr = g_r * cv.x - g_i * cv.y - pv.y, li = g_r * cv.y + g_i * cv.x + pv.x;
        rj.x += lr * x.x - li * x.y;
        rj.y += lr * x.y + li * x.x;
        const double br = g_r * cv.x - g_i * cv.y + pv.y, bi = g_r * cv.y + g_i * cv.x - pv.x;
        rs += sqrt(br * br + bi * bi);
      }
      if (g2v > 0.0) {
        eta = (rj.x * rj.x + rj.y * rj.y) * sqrt(s.g2s[0]) / sqrt(g2v);
        if (a.convention == 1) eta *= sin(th0);
      }
      if (!(isfinite(rj.x) && isfinite(rj.y))) atomicOr(&s.bad, 1);
      const double2 xj = s.xv[j];
      const double xm = sqrt(xj.x * xj.x + xj.y * xj.y);
      // NaN would not order: it is caught by the finiteness test
      if (rs == rs) atomicMax(&s.bnorm_bits, (unsigned long long)__double_as_longlong(rs));
      if (xm == xm) atomicMax(&s.xnorm_bits, (unsigned long long)__double_as_longlong(xm));
    }
    a.intensity[(long long)p * a.ld + j] = eta;
    if (a.rho) a.rho[(long long)p * a.ld + j] = rj;
  }
  __syncthreads();
  // breakdown: ||B||_inf ||B^{-1} e_1||_inf bounds cond_inf(B) from below (as in forward_kernel)
  const bool brk = !(__longlong_as_double((long long)s.bnorm_bits) * __longlong_as_double((long long)s.xnorm_bits) <=
                     BREAKDOWN_COND);
  const int stv = s.flag_singular ? 1 : s.bad ? 2 : brk ? 4 : 0;
  if (stv != 0 && tid < N) {  // a failed pair's outputs are NaN
    a.intensity[(long long)p * a.ld + tid] = NAN;
    if (a.rho) a.rho[(long long)p * a.ld + tid] = make_double2(NAN, NAN);
  }
  if (tid == 0) {
    a.status[p] = stv;
    if (a.nrhst) a.nrhst[p] = nrhst;
  }
}

// The pair list comes ordered by estimated cost, most expensive first;
// rounds of the grid take it in alternating directions (workgroup b gets
// entries b, 2G - 1 - b, 2G + b, ...), which pairs the dearest pairs of one
// round with the cheapest of the next.
template <int STEPPER, bool SAVE>
__global__ __launch_bounds__(LT, 1) void forward_large_kernel(LargeArgs A) {
  char* slot = A.scratch + (long long)blockIdx.x * LSLOT_BYTES;
  const int G = gridDim.x;
#pragma unroll 1
  for (int base = 0, r = 0; base < A.f.n_pairs; base += G, ++r) {
    const int pi = base + ((r & 1) ? G - 1 - (int)blockIdx.x : (int)blockIdx.x);
    if (pi >= A.f.n_pairs) continue;
    const int p = A.f.pair_list ? A.f.pair_list[pi] : pi;
    run_pair<STEPPER, SAVE>(A, p, slot);
    __syncthreads();  // LDS is reused by the next pair
  }
}

}  // namespace

hipError_t launch_forward_large(int stepper, const LargeArgs& a, hipStream_t stream) {
  if (a.f.n_pairs < 1) return hipSuccess;
  const int grid = a.f.n_pairs < a.n_slots ? a.f.n_pairs : a.n_slots;
  if (grid < 1) return hipErrorInvalidValue;
  const bool save = a.f.ws != nullptr;
  if (save && stepper == 2) return hipErrorInvalidValue;  // the splitting stepper keeps no states
  if (stepper == 0 && save)
    hipLaunchKernelGGL((forward_large_kernel<0, true>), dim3(grid), dim3(LT), 0, stream, a);
  else if (stepper == 0)
    hipLaunchKernelGGL((forward_large_kernel<0, false>), dim3(grid), dim3(LT), 0, stream, a);
  else if (stepper == 1 && save)
    hipLaunchKernelGGL((forward_large_kernel<1, true>), dim3(grid), dim3(LT), 0, stream, a);
  else if (stepper == 1)
    hipLaunchKernelGGL((forward_large_kernel<1, false>), dim3(grid), dim3(LT), 0, stream, a);
  else if (stepper == 2)
    hipLaunchKernelGGL((forward_large_kernel<2, false>), dim3(grid), dim3(LT), 0, stream, a);
  else if (stepper == (0 | F32_STAGES) && !save)
    hipLaunchKernelGGL((forward_large_kernel<0 | F32_STAGES, false>), dim3(grid), dim3(LT), 0, stream, a);
  else if (stepper == (1 | F32_STAGES) && !save)
    hipLaunchKernelGGL((forward_large_kernel<1 | F32_STAGES, false>), dim3(grid), dim3(LT), 0, stream, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

int forward_large_slots(int device) {
  int cus = 0, per0 = 0, per1 = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  int per2 = 0;
  int per3 = 0, per4 = 0, per5 = 0, per6 = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per5, forward_large_kernel<0 | F32_STAGES, false>, LT, 0) !=
          hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per6, forward_large_kernel<1 | F32_STAGES, false>, LT, 0) !=
          hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per0, forward_large_kernel<0, false>, LT, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per1, forward_large_kernel<1, false>, LT, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per2, forward_large_kernel<2, false>, LT, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per3, forward_large_kernel<0, true>, LT, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per4, forward_large_kernel<1, true>, LT, 0) != hipSuccess)
    return 0;
  int per = per0 < per1 ? per0 : per1;
  per = per < per2 ? per : per2;
  per = per < per3 ? per : per3;
  per = per < per4 ? per : per4;
  per = per < per5 ? per : per5;
  per = per < per6 ? per : per6;
  return cus * (per > 0 ? per : 0);
}

}  // namespace rheed
