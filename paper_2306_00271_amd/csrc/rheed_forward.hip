// Forward propagation of the many-beam reflection problem on gfx950.
//
// One workgroup (8 waves, two per SIMD) owns one (structure, angle) pair for
// N <= 64 beams, padded to 64.  Of the economical-form state Z = [c; c']
// (Sec. 3.1, Eq. mateq2; the paper's Q-hat and P-hat) the upper block c lives
// in LDS, while c' and the stage products live in registers: wave w holds the
// 16 x 32 block of rows 16 (w & 3) .. +15 and columns 32 (w >> 2) .. +31 of
// every 64 x 64 matrix, laid out as the output of v_mfma_f64_16x16x4f64
// (lane l, value v of J-tile jt -> row 16 (w & 3) + 4v + (l>>4), column
// 32 (w >> 2) + 16 jt + (l&15)), so element e = 4 jt + v of a register matrix
// sits at LDS index ob + 256 v + 16 jt with
// ob = (16 (w & 3) + (l>>4)) 64 + 32 (w >> 2) + (l&15).
//
// One explicit RK step (Sec. 3.4) on y = (c, c'), y' = [[0, I], [-M, 0]] y
// with M(z) = U(z) + Gamma^2, reduces to products G_r = M(z_i + c_r h) X_r
// with stage inputs X_r = c + h c_r c' - h^2 sum_m (A^2)_{rm} G_m, and
//   c  <- c + h c' - h^2 sum_m (bA)_m G_m,   c' <- c' - h sum_m b_m G_m.
// The stages are ordered so that at most three (RK4) or four (RK6) 64 x 64
// matrices are live in registers at any time.  Each product is a complex
// 64 x 64 x 64 GEMM on FP64 MFMA in the 3-real-product form: the B operand is
// the stage input in LDS (the first stage reads c itself), the A operand
// U_{jk} = u_{g_j - g_k} is gathered from the node's rod-difference table in
// LDS (all angles of a structure share these tables; their coupling matrices
// differ only in the diagonal Gamma^2), and each wave runs its two J-tiles
// as six independent accumulation chains.
//
// After every slice the Gershgorin estimate xi of cond(Q) (Sec. 3.2) decides
// the right-hand-side transformation Z <- Z Q^{-1}: T = Q^{-1} by a register-
// resident column Gauss-Jordan elimination with partial pivoting (kept for the
// adjoint), then P <- P T as one more complex GEMM on the matrix cores and
// Q <- I.  The final reflection (Algorithm 1, last lines) inverts
// Gamma Q - iP the same way and applies it to the first column of
// Gamma Q + iP.
#include "rheed_internal.h"
#include "rheed_gj.h"

namespace rheed {

typedef double d4 __attribute__((ext_vector_type(4)));

// J-tiles (16 columns each) per wave: 2 -> 8 waves of 16 rows x 32 columns,
// two waves per SIMD, at most ~216 registers per wave for the RK6 schedule.
constexpr int NJT = 2;
constexpr int NE = 4 * NJT;              // register elements per lane of one 64 x 64 matrix
constexpr int FW = 16 / NJT;             // waves per workgroup
constexpr int FT = FW * 64;              // threads per workgroup

struct Mat {
  double r[NE];
  double i[NE];
};
struct Gidx {  // packed 16-bit table entries of the A operand, two per word
  unsigned v[8];
};
struct G2 {    // Gamma^2 of the lane's four rows
  double v[4];
};

template <int S>
struct Tab;
template <>
struct Tab<0> {  // classical RK4: c = 0, 1/2, 1/2, 1
  static constexpr int nodes = 2;  // distinct c in [0, 1)
  static constexpr int slots = 3;
};
template <>
struct Tab<1> {  // Butcher's 6th order, 7 stages: c = 0, 1/3, 2/3, 1/3, 1/2, 1/2, 1
  static constexpr int nodes = 4;  // 0, 1/3, 1/2, 2/3
  static constexpr int slots = 5;
};
template <>
struct Tab<2> {  // a splitting method: its nodes per slice come with the launch (FwdArgs::sp)
  static constexpr int nodes = 0;
  static constexpr int slots = 5;
};

struct Lds {
  double2 xb[2 * NP * NP];   // [c; X]: c block and stage-input buffer; [Q; P] during eliminations
  double2 tb[5][MAXBOX + 1]; // node tables (Ur, Ui); entry `box` of every row stays 0
  int gj_piv[NP];            // elimination: pivot column of every step,
  int gj_pos[NP];            //   step at which each column was the pivot,
  int gj_cnt;                //   steps published so far
  double g2s[NP];            // Gamma_j^2 (real), 0 on padding
  double bnorm;              // ||Gamma Q - iP||_inf of the reflection solve
  int bhk[NP][2];
  double xo_[4 / NJT][NP];            // per-row sums of |q_ij|, j != i, per column block
  double xdg[4 / NJT][NP];            // per-row |q_ii| partials per column block
  int flag_singular;
};

// The LDS of the one-workgroup kernel.  Every forward kernel of the library
// shares one static LDS allocation (rheed_forward_all.hip), so that a
// launch whose workgroups run pairs of both kinds holds one, not both.
__device__ Lds& fwd_lds_ref();

// top^{-1} for the leading n x n block of the 64 x 64 matrix in s.xb[0 .. NP NP)
// (row major), written back over it (identity outside the n x n block) and,
// with WITH_T, also to t in global memory.  Kept out of line so that its
// registers (the matrix is held in registers during the elimination) do not
// add to those of the RK stages.  The elimination is pipelined over the
// eight waves (gj_inverse_pipe); its step records go to the rows of the
// matrix, which the waves have read by then.
template <bool WITH_T>
__device__ __noinline__ void invert_top(int n, double2* t) {
  Lds& s = fwd_lds_ref();
  constexpr int RB = NP / FW;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double2 za[RB], zs[RB];
#pragma unroll
  for (int m = 0; m < RB; ++m) za[m] = s.xb[(RB * w + m) * NP + lane];
  const int pos = gj_inverse_pipe<FW>(za, zs, n, lane, w, s.xb, s.gj_piv, s.gj_pos, &s.gj_cnt, &s.flag_singular);
#pragma unroll
  for (int m = 0; m < RB; ++m) {
    const int sl = RB * w + m;
    const int row = sl < n ? s.gj_piv[sl] : sl;
    const double2 val = sl < n ? zs[m] : make_double2(pos == sl ? 1.0 : 0.0, 0.0);
    s.xb[row * NP + pos] = val;
    if (WITH_T) t[row * NP + pos] = val;
  }
  __syncthreads();
}

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Element e = 4 jt + v of a wave's register matrix sits at LDS index
// own<LD>(ob, e) of a matrix with row stride LD.
template <int LD>
__device__ __forceinline__ int own(int ob, int e) {
  return ob + 4 * LD * (e & 3) + 16 * (e >> 2);
}

typedef float f4 __attribute__((ext_vector_type(4)));

// Stepper codes of the N <= 64 kernels: bits 0-2 the method (0 RK4, 1 RK6,
// 2 a splitting method), bit 3 set for the lower-precision evaluation, whose
// stage products U X run in FP32 (everything else, the Gamma^2 X term of the
// stages included, stays FP64).
constexpr int F32_STAGES = 8;

// Row of the A operand a lane supplies.  v_mfma_f64_16x16x4f64 returns row
// 4 v + (lane >> 4) of its 16 x 16 result in register v, which the
// epilogues assume; v_mfma_f32_16x16x4f32 returns row 4 (lane >> 4) + v.
// Feeding the FP32 instruction the A rows in the transposed order
// 4 (i & 3) + (i >> 2) (an involution of 0..15) puts row 4 v + (lane >> 4) of
// the product in register v, as for FP64.
template <bool F32>
__device__ __forceinline__ int a_row(int i) {
  return F32 ? 4 * (i & 3) + (i >> 2) : i;
}

// The FP32 form of stage_gemm's U X: the same 3-real-product chains on
// v_mfma_f32_16x16x4f32 (the A rows supplied in a_row<true> order),
// operands rounded to FP32, the chains combined in FP64.
template <int LD, class Epi>
__device__ __forceinline__ void stage_gemm_f32(const double2* __restrict__ xbuf, const double2* __restrict__ tslot,
                                               const unsigned (&gidx)[8], const double (&g2)[4], int ob, int lane,
                                               int cofs, Epi&& epi) {
  __builtin_amdgcn_sched_barrier(0);
  f4 t1[NJT], t2[NJT], t3[NJT];
#pragma unroll
  for (int jt = 0; jt < NJT; ++jt) t1[jt] = t2[jt] = t3[jt] = f4{0, 0, 0, 0};
  const int bb = (lane >> 4) * LD + cofs + (lane & 15);
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const unsigned gi = (q & 1) ? (gidx[q >> 1] >> 16) : (gidx[q >> 1] & 0xffffu);
    const double2 u = tslot[gi];
    const float ur = (float)u.x, ui = (float)u.y, us = (float)(u.x + u.y);
#pragma unroll
    for (int jt = 0; jt < NJT; ++jt) {
      const double2 x = xbuf[bb + 4 * LD * q + 16 * jt];
      t1[jt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ur, (float)x.x, t1[jt], 0, 0, 0);
      t2[jt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ui, (float)x.y, t2[jt], 0, 0, 0);
      t3[jt] = __builtin_amdgcn_mfma_f32_16x16x4f32(us, (float)(x.x + x.y), t3[jt], 0, 0, 0);
    }
    if ((q & 3) == 3) __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int jt = 0; jt < NJT; ++jt) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double2 ov = xbuf[ob + 4 * LD * v + 16 * jt];
      const double a1 = t1[jt][v], a2 = t2[jt][v], a3 = t3[jt][v];
      epi(jt * 4 + v, (a1 - a2) + g2[v] * ov.x, (a3 - a1 - a2) + g2[v] * ov.y);
    }
  }
  __builtin_amdgcn_sched_barrier(0);
}

// G = (U(node) + Gamma^2) X for the wave's 16 x 32 block, X read from LDS
// (row stride LD, the block's columns from cofs); every element of G is
// handed to epi(e, Re G, Im G).  F32: U X in FP32 (stage_gemm_f32).
template <int LD, bool F32 = false, class Epi>
__device__ __forceinline__ void stage_gemm(const double2* __restrict__ xbuf, const double2* __restrict__ tslot,
                                           const unsigned (&gidx)[8], const double (&g2)[4], int ob, int lane,
                                           int cofs, Epi&& epi) {
  if constexpr (F32) {
    stage_gemm_f32<LD>(xbuf, tslot, gidx, g2, ob, lane, cofs, epi);
    return;
  }
  __builtin_amdgcn_sched_barrier(0);
  d4 t1[NJT], t2[NJT], t3[NJT];
#pragma unroll
  for (int jt = 0; jt < NJT; ++jt) t1[jt] = t2[jt] = t3[jt] = d4{0, 0, 0, 0};
  const int bb = (lane >> 4) * LD + cofs + (lane & 15);
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const unsigned gi = (q & 1) ? (gidx[q >> 1] >> 16) : (gidx[q >> 1] & 0xffffu);
    const double2 u = tslot[gi];
    const double us = u.x + u.y;
#pragma unroll
    for (int jt = 0; jt < NJT; ++jt) {
      const double2 x = xbuf[bb + 4 * LD * q + 16 * jt];
      t1[jt] = mfma(u.x, x.x, t1[jt]);
      t2[jt] = mfma(u.y, x.y, t2[jt]);
      t3[jt] = mfma(us, x.x + x.y, t3[jt]);
    }
    if ((q & 3) == 3) __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int jt = 0; jt < NJT; ++jt) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double2 ov = xbuf[ob + 4 * LD * v + 16 * jt];
      epi(jt * 4 + v, (t1[jt][v] - t2[jt][v]) + g2[v] * ov.x, (t3[jt][v] - t1[jt][v] - t2[jt][v]) + g2[v] * ov.y);
    }
  }
  __builtin_amdgcn_sched_barrier(0);
}

// D = A B for 64 x 64 complex A and B in LDS (row major), the wave's 16 x 32
// block of D handed to epi(e, Re D, Im D); 3-real-product form on FP64 MFMA.
template <class Epi>
__device__ __forceinline__ void dense_gemm(const double2* __restrict__ abuf, const double2* __restrict__ bbuf,
                                           int lane, int RT, int CH, Epi&& epi) {
  __builtin_amdgcn_sched_barrier(0);
  d4 t1[NJT], t2[NJT], t3[NJT];
#pragma unroll
  for (int jt = 0; jt < NJT; ++jt) t1[jt] = t2[jt] = t3[jt] = d4{0, 0, 0, 0};
  const int ab = (16 * RT + (lane & 15)) * NP + (lane >> 4);
  const int bb = (lane >> 4) * NP + 16 * NJT * CH + (lane & 15);
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const double2 u = abuf[ab + 4 * q];
    const double us = u.x + u.y;
#pragma unroll
    for (int jt = 0; jt < NJT; ++jt) {
      const double2 x = bbuf[bb + 256 * q + 16 * jt];
      t1[jt] = mfma(u.x, x.x, t1[jt]);
      t2[jt] = mfma(u.y, x.y, t2[jt]);
      t3[jt] = mfma(us, x.x + x.y, t3[jt]);
    }
    if ((q & 3) == 3) __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int jt = 0; jt < NJT; ++jt)
#pragma unroll
    for (int v = 0; v < 4; ++v) epi(jt * 4 + v, t1[jt][v] - t2[jt][v], t3[jt][v] - t1[jt][v] - t2[jt][v]);
  __builtin_amdgcn_sched_barrier(0);
}

#define OWN(e) own<NP>(ob, e)

__device__ __forceinline__ void store_mat(double2* buf, const Mat& m, int ob) {
#pragma unroll
  for (int e = 0; e < NE; ++e) buf[OWN(e)] = make_double2(m.r[e], m.i[e]);
}

// Loads nodes [n0, n1) of a structure's table into their ring slots.
template <int SLOTS, int NT>
__device__ __forceinline__ void load_nodes(Lds& s, const double2* __restrict__ Us, int box, int n0, int n1, int tid) {
  const int total = (n1 - n0) * box;
  for (int e = tid; e < total; e += NT) {
    const int q = e / box;
    const int nn = n0 + q;
    s.tb[nn % SLOTS][e - q * box] = Us[(long long)nn * box + (e - q * box)];
  }
}

// Pair p on one workgroup of FT threads (forward_kernel; also the N <= 64
// pairs of forward_queue_kernel).  BULK: the state starts from a bulk's
// [I; Y] (a.y_bottom) and pairs with a.skip[p] set are not run; the vacuum
// instantiations carry neither.
template <int STEPPER, bool BULK>
__device__ __forceinline__ void small_pair(const FwdArgs& a, int p) {
  using T = Tab<STEPPER & 7>;
  Lds& s = fwd_lds_ref();
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int RT = w & 3, CH = w >> 2;   // row tile, column block of this wave
  if constexpr (BULK) {
    if (a.skip && a.skip[p]) return;
  }
  const StructDev S = a.structs[a.pair_struct[p]];
  const int N = S.n_beams;
  const int L = S.n_slices;
  const double h = S.h;
  const double2* __restrict__ Us = a.U + S.table_off;

  if (tid < NP) {
    s.bhk[tid][0] = tid < N ? a.beams[2 * (S.beam_off + tid)] : 0;
    s.bhk[tid][1] = tid < N ? a.beams[2 * (S.beam_off + tid) + 1] : 0;
  }
  if (tid == 0) s.flag_singular = 0;
  if (tid < T::slots) s.tb[tid][S.box] = make_double2(0.0, 0.0);
  __syncthreads();

  // incidence: b0 = gamma cos(theta0) (cos theta1, sin theta1)
  const double th0 = a.angles[2 * p], th1 = a.angles[2 * p + 1];
  const double b0x = S.gamma * cos(th0) * cos(th1);
  const double b0y = S.gamma * cos(th0) * sin(th1);
  // Gamma_j^2 = gamma^2 - |b0 + k_j|^2 (real; Sec. 2.1, Eq. sch3), 0 on padding
  if (tid < NP) {
    double arg = 0.0;
    if (tid < N) {
      const double qx = b0x + s.bhk[tid][0] * S.recip[0] + s.bhk[tid][1] * S.recip[2];
      const double qy = b0y + s.bhk[tid][0] * S.recip[1] + s.bhk[tid][1] * S.recip[3];
      arg = S.gamma * S.gamma - (qx * qx + qy * qy);
    }
    s.g2s[tid] = arg;
  }
  __syncthreads();
  double g2[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) g2[v] = s.g2s[16 * RT + 4 * v + (lane >> 4)];
  // gather indices of U_{ik} = u_{g_i - g_k} for the A operand of this lane
  unsigned gidx[8];
  {
    const int W = 2 * S.kd + 1;
    const int iA = 16 * RT + a_row<(STEPPER & F32_STAGES) != 0>(lane & 15);
    const int baseA = (s.bhk[iA][0] + S.hd) * W + (s.bhk[iA][1] + S.kd);
#pragma unroll
    for (int q = 0; q < 16; q += 2) {
      const int k0 = 4 * q + (lane >> 4), k1 = 4 * (q + 1) + (lane >> 4);
      const unsigned i0 = (iA < N && k0 < N) ? baseA - (s.bhk[k0][0] * W + s.bhk[k0][1]) : S.box;
      const unsigned i1 = (iA < N && k1 < N) ? baseA - (s.bhk[k1][0] * W + s.bhk[k1][1]) : S.box;
      gidx[q >> 1] = i0 | (i1 << 16);
    }
  }
  double2* cb = s.xb;             // c (upper block of Z), LDS resident
  double2* xb = s.xb + NP * NP;   // stage input X_r
  int ob = (16 * RT + (lane >> 4)) * NP + 16 * NJT * CH + (lane & 15);
  // Z0 = [I; i Gamma]  (spans the same columns as S^{-1}[I; O] of Algorithm 1),
  // or [I; Y] over a bulk whose top state is [I; Y]
  Mat d;
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const int row = 16 * RT + 4 * (e & 3) + (lane >> 4), col = 16 * (NJT * CH + (e >> 2)) + (lane & 15);
    const bool dg = (row == col);
    cb[OWN(e)] = make_double2(dg ? 1.0 : 0.0, 0.0);
    // i Gamma_row with Gamma = sqrt(g2) (open) or -i sqrt(-g2) (evanescent)
    const double g2v = g2[e & 3];
    d.r[e] = (dg && g2v < 0.0) ? sqrt(-g2v) : 0.0;
    d.i[e] = (dg && g2v >= 0.0) ? sqrt(g2v) : 0.0;
    if constexpr (BULK) {
      if (row < N && col < N) {
        const double2 y = a.y_bottom[(long long)p * a.ld * a.ld + row * a.ld + col];
        d.r[e] = y.x;
        d.i[e] = y.y;
      }
    }
  }
  const bool save = a.ws != nullptr;
  char* pws = save ? a.ws + (long long)p * a.ck.pair_stride : nullptr;
  // keep: what the adjoint needs besides the final state (a bulk's layer
  // keeps only the final state)
  bool keep = save;
  if constexpr (BULK) keep = save && !a.final_only;
  int nrhst = 0;

  if constexpr ((STEPPER & 7) != 2) load_nodes<T::slots, FT>(s, Us, S.box, 0, 1, tid);
  // splitting (Sec. 3.4): the slice's node tables sit in ring slots of the
  // stage-input buffer, which the splitting steps do not otherwise use (the
  // transformation below overwrites it, so they are loaded every slice)
  auto load_ring = [&](int n0, int count) {
    const int total = count * (S.box + 1);
    for (int e = tid; e < total; e += FT) {
      const int m = e / (S.box + 1), j = e - m * (S.box + 1);
      xb[m * (MAXBOX + 1) + j] = j < S.box ? Us[(long long)(n0 + m) * S.box + j] : make_double2(0.0, 0.0);
    }
    __syncthreads();
  };
  // kick: c' -= h w (U + Gamma^2) c with the table in ring slot m; c is read
  // by every wave, so a barrier follows before anything writes it
  auto kick = [&](int m, double wgt) {
    stage_gemm<NP, (STEPPER & F32_STAGES) != 0>(cb, xb + m * (MAXBOX + 1), gidx, g2, ob, lane, 16 * NJT * CH, [&](int e, double gr, double gi) {
      d.r[e] -= h * wgt * gr;
      d.i[e] -= h * wgt * gi;
    });
    __syncthreads();
  };
  // drift: c += h w c' (each lane its own elements), then a barrier before c is read
  auto drift = [&](double wgt) {
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      double2 cv = cb[OWN(e)];
      cv.x += h * wgt * d.r[e];
      cv.y += h * wgt * d.i[e];
      cb[OWN(e)] = cv;
    }
    __syncthreads();
  };
  for (int i = 0; i < L; ++i) {
    // keep the address base from being expanded into loop-invariant registers
    asm volatile("" : "+v"(ob));
    if (keep && (i % a.ck.every) == 0) {
      double2* st = reinterpret_cast<double2*>(pws + (long long)(i / a.ck.every) * a.ck.state_bytes);
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        st[OWN(e)] = cb[OWN(e)];
        st[NP * NP + OWN(e)] = make_double2(d.r[e], d.i[e]);
      }
    }
    const int nb = i * T::nodes;  // node index of c = 0 in this slice
    if constexpr ((STEPPER & 7) != 2) load_nodes<T::slots, FT>(s, Us, S.box, nb + 1, nb + T::nodes + 1, tid);
    const double hh = h * h;
    if constexpr ((STEPPER & 7) == 2) {
      const SplitSteps& sp = a.sp;
      load_ring(i * sp.nps, sp.nps);
      if (sp.form == 0) {
        // BAB; the previous slice's last kick (at this slice's start) is merged
        // into this slice's first: kicks change c' only, so the badness and
        // the transformation (a right multiplication) are unaffected
        kick(sp.node[0], i == 0 ? sp.b[0] : sp.b[0] + sp.b[sp.kicks - 1]);
        for (int r = 0; r + 1 < sp.kicks; ++r) {
          drift(sp.a[r]);
          if (r + 2 < sp.kicks) kick(sp.node[r + 1], sp.b[r + 1]);
        }
      } else {
        // ABA
        drift(sp.a[0]);
        for (int r = 0; r < sp.kicks; ++r) {
          kick(sp.node[r], sp.b[r]);
          drift(sp.a[r + 1]);
        }
      }
    } else if constexpr ((STEPPER & 7) == 0) {
      const double2* t0 = s.tb[nb % 3];
      const double2* th = s.tb[(nb + 1) % 3];
      const double2* t1 = s.tb[(nb + 2) % 3];
      // X1 = c (read in place), X2 = c + h/2 c'
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const double2 cv = cb[OWN(e)];
        xb[OWN(e)] = make_double2(cv.x + 0.5 * h * d.r[e], cv.y + 0.5 * h * d.i[e]);
      }
      __syncthreads();
      Mat G1, G2;
      stage_gemm<NP, (STEPPER & F32_STAGES) != 0>(cb, t0, gidx, g2, ob, lane, 16 * NJT * CH, [&](int e, double gr, double gi) { G1.r[e] = gr; G1.i[e] = gi; });
      stage_gemm<NP, (STEPPER & F32_STAGES) != 0>(xb, th, gidx, g2, ob, lane, 16 * NJT * CH, [&](int e, double gr, double gi) { G2.r[e] = gr; G2.i[e] = gi; });
      __syncthreads();
      // X3 = c + h/2 c' - h^2/4 G1 -> LDS;  X4 = c + h c' - h^2/2 G2 (kept in G1);
      // c <- c + h c' - h^2/6 (G1 + G2);  c' <- c' - h/6 (G1 + 2 G2)
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const double2 cv = cb[OWN(e)];
        const double dr = d.r[e], di = d.i[e];
        const double g1r = G1.r[e], g1i = G1.i[e], g2r = G2.r[e], g2i = G2.i[e];
        xb[OWN(e)] = make_double2(cv.x + 0.5 * h * dr - 0.25 * hh * g1r, cv.y + 0.5 * h * di - 0.25 * hh * g1i);
        G1.r[e] = cv.x + h * dr - 0.5 * hh * g2r;
        G1.i[e] = cv.y + h * di - 0.5 * hh * g2i;
        cb[OWN(e)] = make_double2(cv.x + h * dr - (hh / 6.0) * (g1r + g2r), cv.y + h * di - (hh / 6.0) * (g1i + g2i));
        d.r[e] = dr - (h / 6.0) * (g1r + 2.0 * g2r);
        d.i[e] = di - (h / 6.0) * (g1i + 2.0 * g2i);
      }
      __syncthreads();
      stage_gemm<NP, (STEPPER & F32_STAGES) != 0>(xb, th, gidx, g2, ob, lane, 16 * NJT * CH, [&](int e, double gr, double gi) {  // G3
        double2 cv = cb[OWN(e)];
        cv.x -= (hh / 6.0) * gr;
        cv.y -= (hh / 6.0) * gi;
        cb[OWN(e)] = cv;
        d.r[e] -= (h / 3.0) * gr;
        d.i[e] -= (h / 3.0) * gi;
      });
      __syncthreads();
      store_mat(xb, G1, ob);  // X4
      __syncthreads();
      stage_gemm<NP, (STEPPER & F32_STAGES) != 0>(xb, t1, gidx, g2, ob, lane, 16 * NJT * CH, [&](int e, double gr, double gi) {  // G4
        d.r[e] -= (h / 6.0) * gr;
        d.i[e] -= (h / 6.0) * gi;
      });
    } else {
      const double2* tA = s.tb[nb % 5];        // c = 0
      const double2* tB = s.tb[(nb + 1) % 5];  // c = 1/3
      const double2* tC = s.tb[(nb + 2) % 5];  // c = 1/2
      const double2* tD = s.tb[(nb + 3) % 5];  // c = 2/3
      const double2* tE = s.tb[(nb + 4) % 5];  // c = 1
      // X1 = c (read in place), X2 = c + h/3 c'
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const double2 cv = cb[OWN(e)];
        xb[OWN(e)] = make_double2(cv.x + (h / 3.0) * d.r[e], cv.y + (h / 3.0) * d.i[e]);
      }
      __syncthreads();
      Mat G1, G2, G3;
      stage_gemm<NP, (STEPPER & F32_STAGES) != 0>(cb, tA, gidx, g2, ob, lane, 16 * NJT * CH, [&](int e, double gr, double gi) { G1.r[e] = gr; G1.i[e] = gi; });
      stage_gemm<NP, (STEPPER & F32_STAGES) != 0>(xb, tB, gidx, g2, ob, lane, 16 * NJT * CH, [&](int e, double gr, double gi) { G2.r[e] = gr; G2.i[e] = gi; });
      __syncthreads();
      // X3 = c + 2h/3 c' - h^2 (2/9) G1
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const double2 cv = cb[OWN(e)];
        xb[OWN(e)] = make_double2(cv.x + (2.0 * h / 3.0) * d.r[e] - hh * (2.0 / 9.0) * G1.r[e],
                                  cv.y + (2.0 * h / 3.0) * d.i[e] - hh * (2.0 / 9.0) * G1.i[e]);
      }
      __syncthreads();
      stage_gemm<NP, (STEPPER & F32_STAGES) != 0>(xb, tD, gidx, g2, ob, lane, 16 * NJT * CH, [&](int e, double gr, double gi) { G3.r[e] = gr; G3.i[e] = gi; });
      __syncthreads();
      // X4 = c + h/3 c' - h^2 (G1/9 - G2/18)
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const double2 cv = cb[OWN(e)];
        xb[OWN(e)] = make_double2(cv.x + (h / 3.0) * d.r[e] - hh * ((1.0 / 9.0) * G1.r[e] - (1.0 / 18.0) * G2.r[e]),
                                  cv.y + (h / 3.0) * d.i[e] - hh * ((1.0 / 9.0) * G1.i[e] - (1.0 / 18.0) * G2.i[e]));
      }
      __syncthreads();
      // G4; per element {c, c', G1, G2, G3, G4} -> X5, X6, T7, c-partial (LDS), c'-partial
      Mat& X5 = G1;
      Mat& X6 = G2;
      Mat& T7 = G3;
      stage_gemm<NP, (STEPPER & F32_STAGES) != 0>(xb, tB, gidx, g2, ob, lane, 16 * NJT * CH, [&](int e, double a4, double b4) {
        const double2 cv = cb[OWN(e)];
        const double dr = d.r[e], di = d.i[e];
        const double a1 = G1.r[e], b1 = G1.i[e], a2 = G2.r[e], b2 = G2.i[e], a3 = G3.r[e], b3 = G3.i[e];
        X5.r[e] = cv.x + 0.5 * h * dr - hh * ((11.0 / 32.0) * a1 - 0.25 * a2 + (1.0 / 32.0) * a3);
        X5.i[e] = cv.y + 0.5 * h * di - hh * ((11.0 / 32.0) * b1 - 0.25 * b2 + (1.0 / 32.0) * b3);
        X6.r[e] = cv.x + 0.5 * h * dr - hh * ((9.0 / 32.0) * a1 + (1.0 / 16.0) * a2 - (1.0 / 32.0) * a3 - (3.0 / 16.0) * a4);
        X6.i[e] = cv.y + 0.5 * h * di - hh * ((9.0 / 32.0) * b1 + (1.0 / 16.0) * b2 - (1.0 / 32.0) * b3 - (3.0 / 16.0) * b4);
        T7.r[e] = cv.x + h * dr - hh * ((-3.0 / 22.0) * a1 - (3.0 / 22.0) * a2 + (9.0 / 22.0) * a3 + (12.0 / 11.0) * a4);
        T7.i[e] = cv.y + h * di - hh * ((-3.0 / 22.0) * b1 - (3.0 / 22.0) * b2 + (9.0 / 22.0) * b3 + (12.0 / 11.0) * b4);
        cb[OWN(e)] = make_double2(cv.x + h * dr - hh * ((11.0 / 120.0) * a1 + (9.0 / 40.0) * a3 + (9.0 / 20.0) * a4),
                                  cv.y + h * di - hh * ((11.0 / 120.0) * b1 + (9.0 / 40.0) * b3 + (9.0 / 20.0) * b4));
        d.r[e] = dr - h * ((11.0 / 120.0) * a1 + (27.0 / 40.0) * a3 + (27.0 / 40.0) * a4);
        d.i[e] = di - h * ((11.0 / 120.0) * b1 + (27.0 / 40.0) * b3 + (27.0 / 40.0) * b4);
      });
      __syncthreads();
      store_mat(xb, X5, ob);
      __syncthreads();
      stage_gemm<NP, (STEPPER & F32_STAGES) != 0>(xb, tC, gidx, g2, ob, lane, 16 * NJT * CH, [&](int e, double gr, double gi) {  // G5
        T7.r[e] += hh * (8.0 / 11.0) * gr;
        T7.i[e] += hh * (8.0 / 11.0) * gi;
        double2 cv = cb[OWN(e)];
        cv.x += hh * (2.0 / 15.0) * gr;
        cv.y += hh * (2.0 / 15.0) * gi;
        cb[OWN(e)] = cv;
        d.r[e] += h * (4.0 / 15.0) * gr;
        d.i[e] += h * (4.0 / 15.0) * gi;
      });
      __syncthreads();
      store_mat(xb, X6, ob);
      __syncthreads();
      stage_gemm<NP, (STEPPER & F32_STAGES) != 0>(xb, tC, gidx, g2, ob, lane, 16 * NJT * CH, [&](int e, double gr, double gi) {  // G6
        double2 cv = cb[OWN(e)];
        cv.x += hh * (2.0 / 15.0) * gr;
        cv.y += hh * (2.0 / 15.0) * gi;
        cb[OWN(e)] = cv;
        d.r[e] += h * (4.0 / 15.0) * gr;
        d.i[e] += h * (4.0 / 15.0) * gi;
      });
      __syncthreads();
      store_mat(xb, T7, ob);  // X7
      __syncthreads();
      stage_gemm<NP, (STEPPER & F32_STAGES) != 0>(xb, tE, gidx, g2, ob, lane, 16 * NJT * CH, [&](int e, double gr, double gi) {  // G7
        d.r[e] -= h * (11.0 / 120.0) * gr;
        d.i[e] -= h * (11.0 / 120.0) * gi;
      });
    }

    // condition estimate of Q = c over rows/cols < N (Sec. 3.2): the
    // Gershgorin / Varah bound max(|q_ii| + r_i) / min(|q_ii| - r_i)
    {
      double dg[4] = {0, 0, 0, 0}, of[4] = {0, 0, 0, 0};
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const int row = 16 * RT + 4 * (e & 3) + (lane >> 4), col = 16 * (NJT * CH + (e >> 2)) + (lane & 15);
        const double2 cv = cb[OWN(e)];
        const double av = sqrt(cv.x * cv.x + cv.y * cv.y);
        if (row < N && col < N) {
          if (row == col) dg[e & 3] += av;
          else of[e & 3] += av;
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
          dg[v] += __shfl_xor(dg[v], off, 64);
          of[v] += __shfl_xor(of[v], off, 64);
        }
      }
      if ((lane & 15) == 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * RT + 4 * v + (lane >> 4);
          s.xdg[CH][row] = dg[v];
          s.xo_[CH][row] = of[v];
        }
      }
    }
    __syncthreads();
    bool do_rhst;
    {
      double dgl = 0.0, ofl = 0.0;
#pragma unroll
      for (int c2 = 0; c2 < 4 / NJT; ++c2) {
        dgl += s.xdg[c2][lane];
        ofl += s.xo_[c2][lane];
      }
      double hi = lane < N ? dgl + ofl : 0.0;
      double lo = lane < N ? dgl - ofl : 1.0e308;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        hi = fmax(hi, __shfl_xor(hi, off, 64));
        lo = fmin(lo, __shfl_xor(lo, off, 64));
      }
      const double xi = lo > 0.0 ? hi / lo : INFINITY;
      do_rhst = xi > a.threshold;
    }
    if (keep && tid == 0) pws[a.ck.flags_off + i] = do_rhst ? 1 : 0;
    if (do_rhst) {
      // Z <- Z Q^{-1}: T = Q^{-1} by elimination (kept for the adjoint when
      // saving), then P <- P T on the matrix cores, c <- I
      ++nrhst;
      store_mat(xb, d, ob);
      __syncthreads();
      if (keep)
        invert_top<true>(N, reinterpret_cast<double2*>(pws + a.ck.q_off + (long long)i * NP * NP * sizeof(double2)));
      else
        invert_top<false>(N, nullptr);
      dense_gemm(xb, cb, lane, RT, CH, [&](int e, double gr, double gi) {
        d.r[e] = gr;
        d.i[e] = gi;
      });
      if (keep && a.ck.r_off) {  // R = P Q^{-1} for an adjoint that keeps states only every few slices
        double2* rs = reinterpret_cast<double2*>(pws + a.ck.r_off + (long long)i * NP * NP * sizeof(double2));
#pragma unroll
        for (int e = 0; e < NE; ++e) rs[OWN(e)] = make_double2(d.r[e], d.i[e]);
      }
      __syncthreads();
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const int row = 16 * RT + 4 * (e & 3) + (lane >> 4), col = 16 * (NJT * CH + (e >> 2)) + (lane & 15);
        cb[OWN(e)] = make_double2((row == col) ? 1.0 : 0.0, 0.0);
      }
    }
    __syncthreads();
  }
  if constexpr ((STEPPER & 7) == 2) {
    if (a.sp.form == 0) {  // BAB: the last slice's final kick, at z = 0 (node L nps)
      load_ring(L * a.sp.nps, 1);
      kick(0, a.sp.b[a.sp.kicks - 1]);
    }
  }

  if (save) {
    double2* st = reinterpret_cast<double2*>(pws + (long long)(a.ck.max_ckpt - 1) * a.ck.state_bytes);
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      st[OWN(e)] = cb[OWN(e)];
      st[NP * NP + OWN(e)] = make_double2(d.r[e], d.i[e]);
    }
  }
  // reflection: Z <- S Z = [Gamma Q - iP; Gamma Q + iP]; R = lower upper^{-1};
  // rho = R e_1 = lower (upper^{-1} e_1)
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const double2 cv = cb[OWN(e)];
    const double g2v = g2[e & 3];
    const double g_r = g2v >= 0.0 ? sqrt(g2v) : 0.0, g_i = g2v >= 0.0 ? 0.0 : -sqrt(-g2v);
    const double qr = g_r * cv.x - g_i * cv.y;
    const double qi = g_r * cv.y + g_i * cv.x;
    // -iP = (P.i, -P.r);  +iP = (-P.i, P.r)
    cb[OWN(e)] = make_double2(qr + d.i[e], qi - d.r[e]);
    xb[OWN(e)] = make_double2(qr - d.i[e], qi + d.r[e]);
  }
  __syncthreads();
  // ||Gamma Q - iP||_inf, for the breakdown test below (wave 0: one row per lane)
  if (w == 0) {
    double rs = 0.0;
    if (lane < N)
      for (int k = 0; k < N; ++k) {
        const double2 v = cb[lane * NP + k];
        rs += sqrt(v.x * v.x + v.y * v.y);
      }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) rs = fmax(rs, __shfl_xor(rs, off, 64));
    if (lane == 0) s.bnorm = rs;
  }
  invert_top<false>(N, nullptr);
  if (tid < NP) {
    const int j = tid;
    double eta = 0.0;
    double2 rj = make_double2(0.0, 0.0);
    // breakdown: ||B||_inf ||B^{-1} e_1||_inf bounds cond_inf(B) from below; past
    // BREAKDOWN_COND the reflection solve has lost every digit the paper's
    // assumption (the inverses exist) relies on
    double xm = 0.0;
    if (j < N) {
      const double2 x = cb[j * NP];
      xm = sqrt(x.x * x.x + x.y * x.y);
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) xm = fmax(xm, __shfl_xor(xm, off, 64));
    const bool brk = !(s.bnorm * xm <= BREAKDOWN_COND);
    if (j < N) {
      for (int k = 0; k < N; ++k) {
        const double2 l = xb[j * NP + k], x = cb[k * NP];
        rj.x += l.x * x.x - l.y * x.y;
        rj.y += l.x * x.y + l.y * x.x;
      }
      const double g00 = s.g2s[0];
      const double gj = s.g2s[j];
      if (gj > 0.0) {
        eta = (rj.x * rj.x + rj.y * rj.y) * sqrt(g00) / sqrt(gj);
        if (a.convention == 1) eta *= sin(th0);
      }
    }
    const bool fin = isfinite(rj.x) && isfinite(rj.y);
    const unsigned long long bad = __ballot(!fin);
    int st = 0;
    if (s.flag_singular) st = 1;
    else if (bad) st = 2;
    else if (brk) st = 4;
    if (st != 0 && j < N) {  // a failed pair's outputs are NaN
      eta = NAN;
      rj = make_double2(NAN, NAN);
    }
    if (j < a.ld) {
      a.intensity[(long long)p * a.ld + j] = eta;
      if (a.rho) a.rho[(long long)p * a.ld + j] = rj;
    }
    for (int jt = NP + j; jt < a.ld; jt += NP) {  // outputs of a wider plan's padding
      a.intensity[(long long)p * a.ld + jt] = 0.0;
      if (a.rho) a.rho[(long long)p * a.ld + jt] = make_double2(0.0, 0.0);
    }
    if (j == 0) {
      a.status[p] = st;
      if (a.nrhst) a.nrhst[p] = nrhst;
    }
  }
}

template <int STEPPER, bool BULK>
__global__ __launch_bounds__(FT, 1) void forward_kernel(FwdArgs a) {
  small_pair<STEPPER, BULK>(a, a.pair_list ? a.pair_list[blockIdx.x] : blockIdx.x);
}
#undef OWN


template <int LD>
__device__ __forceinline__ void store_mat_ld(double2* buf, const Mat& m, int ob) {
#pragma unroll
  for (int e = 0; e < NE; ++e) buf[own<LD>(ob, e)] = make_double2(m.r[e], m.i[e]);
}

// One explicit RK step of the slice on (c, c'): c in LDS (cb), c' in
// registers (d), stage inputs through xb; the slice's node tables (the c
// values of Tab<STEPPER>, then the next slice's c = 0) are ring slots
// (nb + q) % slots of tb0, each MAXBOX + 1 entries.  LD is the LDS
// row stride of cb and xb, cofs the column offset of this wave's block.
template <int STEPPER, int LD>
__device__ __forceinline__ Mat rk_slice(double2* cb, double2* xb, const double2* tb0, int nb, const Gidx gx,
                                        const G2 gg, int ob, int lane, int cofs, double h, Mat d) {
  constexpr int SL = Tab<STEPPER & 7>::slots;
  unsigned gidx[8];
  double g2[4];
#pragma unroll
  for (int q = 0; q < 8; ++q) gidx[q] = gx.v[q];
#pragma unroll
  for (int q = 0; q < 4; ++q) g2[q] = gg.v[q];
const double hh = h * h;
  if constexpr ((STEPPER & 7) == 0) {
    const double2* t0 = tb0 + (nb % SL) * (MAXBOX + 1);
    const double2* th = tb0 + ((nb + 1) % SL) * (MAXBOX + 1);
    const double2* t1 = tb0 + ((nb + 2) % SL) * (MAXBOX + 1);
    // X1 = c (read in place), X2 = c + h/2 c'
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const double2 cv = cb[own<LD>(ob, e)];
      xb[own<LD>(ob, e)] = make_double2(cv.x + 0.5 * h * d.r[e], cv.y + 0.5 * h * d.i[e]);
    }
    __syncthreads();
    Mat G1, G2;
    stage_gemm<LD, (STEPPER & F32_STAGES) != 0>(cb, t0, gidx, g2, ob, lane, cofs, [&](int e, double gr, double gi) { G1.r[e] = gr; G1.i[e] = gi; });
    stage_gemm<LD, (STEPPER & F32_STAGES) != 0>(xb, th, gidx, g2, ob, lane, cofs, [&](int e, double gr, double gi) { G2.r[e] = gr; G2.i[e] = gi; });
    __syncthreads();
    // X3 = c + h/2 c' - h^2/4 G1 -> LDS;  X4 = c + h c' - h^2/2 G2 (kept in G1);
    // c <- c + h c' - h^2/6 (G1 + G2);  c' <- c' - h/6 (G1 + 2 G2)
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const double2 cv = cb[own<LD>(ob, e)];
      const double dr = d.r[e], di = d.i[e];
      const double g1r = G1.r[e], g1i = G1.i[e], g2r = G2.r[e], g2i = G2.i[e];
      xb[own<LD>(ob, e)] = make_double2(cv.x + 0.5 * h * dr - 0.25 * hh * g1r, cv.y + 0.5 * h * di - 0.25 * hh * g1i);
      G1.r[e] = cv.x + h * dr - 0.5 * hh * g2r;
      G1.i[e] = cv.y + h * di - 0.5 * hh * g2i;
      cb[own<LD>(ob, e)] = make_double2(cv.x + h * dr - (hh / 6.0) * (g1r + g2r), cv.y + h * di - (hh / 6.0) * (g1i + g2i));
      d.r[e] = dr - (h / 6.0) * (g1r + 2.0 * g2r);
      d.i[e] = di - (h / 6.0) * (g1i + 2.0 * g2i);
    }
    __syncthreads();
    stage_gemm<LD, (STEPPER & F32_STAGES) != 0>(xb, th, gidx, g2, ob, lane, cofs, [&](int e, double gr, double gi) {  // G3
      double2 cv = cb[own<LD>(ob, e)];
      cv.x -= (hh / 6.0) * gr;
      cv.y -= (hh / 6.0) * gi;
      cb[own<LD>(ob, e)] = cv;
      d.r[e] -= (h / 3.0) * gr;
      d.i[e] -= (h / 3.0) * gi;
    });
    __syncthreads();
    store_mat_ld<LD>(xb, G1, ob);  // X4
    __syncthreads();
    stage_gemm<LD, (STEPPER & F32_STAGES) != 0>(xb, t1, gidx, g2, ob, lane, cofs, [&](int e, double gr, double gi) {  // G4
      d.r[e] -= (h / 6.0) * gr;
      d.i[e] -= (h / 6.0) * gi;
    });
  } else {
    const double2* tA = tb0 + (nb % SL) * (MAXBOX + 1);        // c = 0
    const double2* tB = tb0 + ((nb + 1) % SL) * (MAXBOX + 1);  // c = 1/3
    const double2* tC = tb0 + ((nb + 2) % SL) * (MAXBOX + 1);  // c = 1/2
    const double2* tD = tb0 + ((nb + 3) % SL) * (MAXBOX + 1);  // c = 2/3
    const double2* tE = tb0 + ((nb + 4) % SL) * (MAXBOX + 1);  // c = 1
    // X1 = c (read in place), X2 = c + h/3 c'
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const double2 cv = cb[own<LD>(ob, e)];
      xb[own<LD>(ob, e)] = make_double2(cv.x + (h / 3.0) * d.r[e], cv.y + (h / 3.0) * d.i[e]);
    }
    __syncthreads();
    Mat G1, G2, G3;
    stage_gemm<LD, (STEPPER & F32_STAGES) != 0>(cb, tA, gidx, g2, ob, lane, cofs, [&](int e, double gr, double gi) { G1.r[e] = gr; G1.i[e] = gi; });
    stage_gemm<LD, (STEPPER & F32_STAGES) != 0>(xb, tB, gidx, g2, ob, lane, cofs, [&](int e, double gr, double gi) { G2.r[e] = gr; G2.i[e] = gi; });
    __syncthreads();
    // X3 = c + 2h/3 c' - h^2 (2/9) G1
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const double2 cv = cb[own<LD>(ob, e)];
      xb[own<LD>(ob, e)] = make_double2(cv.x + (2.0 * h / 3.0) * d.r[e] - hh * (2.0 / 9.0) * G1.r[e],
                                cv.y + (2.0 * h / 3.0) * d.i[e] - hh * (2.0 / 9.0) * G1.i[e]);
    }
    __syncthreads();
    stage_gemm<LD, (STEPPER & F32_STAGES) != 0>(xb, tD, gidx, g2, ob, lane, cofs, [&](int e, double gr, double gi) { G3.r[e] = gr; G3.i[e] = gi; });
    __syncthreads();
    // X4 = c + h/3 c' - h^2 (G1/9 - G2/18)
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const double2 cv = cb[own<LD>(ob, e)];
      xb[own<LD>(ob, e)] = make_double2(cv.x + (h / 3.0) * d.r[e] - hh * ((1.0 / 9.0) * G1.r[e] - (1.0 / 18.0) * G2.r[e]),
                                cv.y + (h / 3.0) * d.i[e] - hh * ((1.0 / 9.0) * G1.i[e] - (1.0 / 18.0) * G2.i[e]));
    }
    __syncthreads();
    // G4; per element {c, c', G1, G2, G3, G4} -> X5, X6, T7, c-partial (LDS), c'-partial
    Mat& X5 = G1;
    Mat& X6 = G2;
    Mat& T7 = G3;
    stage_gemm<LD, (STEPPER & F32_STAGES) != 0>(xb, tB, gidx, g2, ob, lane, cofs, [&](int e, double a4, double b4) {
      const double2 cv = cb[own<LD>(ob, e)];
      const double dr = d.r[e], di = d.i[e];
      const double a1 = G1.r[e], b1 = G1.i[e], a2 = G2.r[e], b2 = G2.i[e], a3 = G3.r[e], b3 = G3.i[e];
      X5.r[e] = cv.x + 0.5 * h * dr - hh * ((11.0 / 32.0) * a1 - 0.25 * a2 + (1.0 / 32.0) * a3);
      X5.i[e] = cv.y + 0.5 * h * di - hh * ((11.0 / 32.0) * b1 - 0.25 * b2 + (1.0 / 32.0) * b3);
      X6.r[e] = cv.x + 0.5 * h * dr - hh * ((9.0 / 32.0) * a1 + (1.0 / 16.0) * a2 - (1.0 / 32.0) * a3 - (3.0 / 16.0) * a4);
      X6.i[e] = cv.y + 0.5 * h * di - hh * ((9.0 / 32.0) * b1 + (1.0 / 16.0) * b2 - (1.0 / 32.0) * b3 - (3.0 / 16.0) * b4);
      T7.r[e] = cv.x + h * dr - hh * ((-3.0 / 22.0) * a1 - (3.0 / 22.0) * a2 + (9.0 / 22.0) * a3 + (12.0 / 11.0) * a4);
      T7.i[e] = cv.y + h * di - hh * ((-3.0 / 22.0) * b1 - (3.0 / 22.0) * b2 + (9.0 / 22.0) * b3 + (12.0 / 11.0) * b4);
      cb[own<LD>(ob, e)] = make_double2(cv.x + h * dr - hh * ((11.0 / 120.0) * a1 + (9.0 / 40.0) * a3 + (9.0 / 20.0) * a4),
                                cv.y + h * di - hh * ((11.0 / 120.0) * b1 + (9.0 / 40.0) * b3 + (9.0 / 20.0) * b4));
      d.r[e] = dr - h * ((11.0 / 120.0) * a1 + (27.0 / 40.0) * a3 + (27.0 / 40.0) * a4);
      d.i[e] = di - h * ((11.0 / 120.0) * b1 + (27.0 / 40.0) * b3 + (27.0 / 40.0) * b4);
    });
    __syncthreads();
    store_mat_ld<LD>(xb, X5, ob);
    __syncthreads();
    stage_gemm<LD, (STEPPER & F32_STAGES) != 0>(xb, tC, gidx, g2, ob, lane, cofs, [&](int e, double gr, double gi) {  // G5
      T7.r[e] += hh * (8.0 / 11.0) * gr;
      T7.i[e] += hh * (8.0 / 11.0) * gi;
      double2 cv = cb[own<LD>(ob, e)];
      cv.x += hh * (2.0 / 15.0) * gr;
      cv.y += hh * (2.0 / 15.0) * gi;
      cb[own<LD>(ob, e)] = cv;
      d.r[e] += h * (4.0 / 15.0) * gr;
      d.i[e] += h * (4.0 / 15.0) * gi;
    });
    __syncthreads();
    store_mat_ld<LD>(xb, X6, ob);
    __syncthreads();
    stage_gemm<LD, (STEPPER & F32_STAGES) != 0>(xb, tC, gidx, g2, ob, lane, cofs, [&](int e, double gr, double gi) {  // G6
      double2 cv = cb[own<LD>(ob, e)];
      cv.x += hh * (2.0 / 15.0) * gr;
      cv.y += hh * (2.0 / 15.0) * gi;
      cb[own<LD>(ob, e)] = cv;
      d.r[e] += h * (4.0 / 15.0) * gr;
      d.i[e] += h * (4.0 / 15.0) * gi;
    });
    __syncthreads();
    store_mat_ld<LD>(xb, T7, ob);  // X7
    __syncthreads();
    stage_gemm<LD, (STEPPER & F32_STAGES) != 0>(xb, tE, gidx, g2, ob, lane, cofs, [&](int e, double gr, double gi) {  // G7
      d.r[e] -= h * (11.0 / 120.0) * gr;
      d.i[e] -= h * (11.0 / 120.0) * gi;
    });
  }
  return d;
}


// ---------------------------------------------------------------------------
// Split launch: two workgroups of four waves per pair (one per SIMD, so each
// wave has the whole register file of its SIMD), each owning 32 of the 64
// columns of Z.  The RK stages act on columns independently, so each half
// steps its own columns; what couples the columns goes through a per-pair
// exchange block in global memory: the badness partials (row sums over each
// half's columns) after every slice, and the halves of [Q; P] at every
// right-hand-side transformation and before the reflection solve.  Both
// halves combine the partials in the same order, so they take the same
// decisions; at a transformation both invert the whole Q (the elimination is
// latency-bound, so the redundant work costs no time) and multiply P by the
// columns of Q^{-1} they own.  A launch needs both halves of every pair
// resident at once (cooperative launch), which holds up to one pair per two
// CUs; a bounded wait marks the pair RHEED_PAIR_SYNC instead of hanging.
// ---------------------------------------------------------------------------

constexpr int SW = 4;        // waves per half-pair workgroup
constexpr int ST = SW * 64;  // threads per half-pair workgroup
constexpr int HC = NP / 2;   // columns per half

struct SplitLds {
  double2 cx[2 * NP * HC];   // c of this half [NP][HC], then the stage input [NP][HC]; [NP][NP] at the end
  double2 ext[NP * NP];      // Q of both halves for the elimination, then Q^{-1}
  double2 tb[5][MAXBOX + 1];
  int gj_piv[NP];            // pivot column of every elimination step
  int gj_pos[NP];            // step at which each column was the pivot
  int gj_cnt;                // elimination steps published so far
  double g2s[NP];
  double bnorm;              // ||Gamma Q - iP||_inf of the reflection solve
  int bhk[NP][2];
  double xi_loc[2][NP];      // this half's |q_rr| and sum_{j != r} |q_rj| per row
  int flag_singular;
  int sync_fail;
};

__shared__ SplitLds split_lds;

constexpr int XCH_SPIN = 1 << 22;  // polls before a wait gives up

// Exchange protocol.  Data goes through memory as agent-scope atomic
// accesses (coherent across the XCDs' L2 caches).  A writer makes its
// stores complete (each wave), synchronises its workgroup, and raises its
// counter with an agent-scope release store, which writes the L2 back first,
// so the data is in memory before the counter is.  A reader polls the
// partner's counter with coherent loads and then reads the data, issued
// after the counter was seen.
__device__ __forceinline__ void xput(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double xget(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void xput2(double2* p, double2 v) {
  xput(&p->x, v.x);
  xput(&p->y, v.y);
}
__device__ __forceinline__ double2 xget2(const double2* p) {
  return make_double2(xget(&p->x), xget(&p->y));
}

// Raises this workgroup's counter to v once its exchange stores are in memory.
__device__ __forceinline__ void xch_publish(unsigned long long* cnt, unsigned long long v) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's stores have reached the L2
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(cnt, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits until the partner's counter reaches v.  A wait gives up after about
// XCH_TICKS of the constant-rate clock (far beyond any legitimate skew between
// the halves) and sets *fail; after that, later waits return at once.  A
// half that gives up also writes the launch number to its failure word in the
// exchange block (before any later counter raise, which releases it), so that
// half 0, which writes the pair's status, reports the pair whichever half
// lost contact.  give_up (set from the host to test this path) makes the
// first wait fail without polling.
constexpr long long XCH_TICKS = 2000000;
__device__ __forceinline__ void xch_wait(unsigned long long* cnt, unsigned long long v, int* fail,
                                         unsigned long long* fail_word, unsigned long long epoch, bool give_up) {
  if (threadIdx.x == 0 && !*fail) {
    const long long t0 = wall_clock64();
    int it = 0;
    while (give_up || __hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < v) {
      if (give_up || ++it > XCH_SPIN || wall_clock64() - t0 > XCH_TICKS) {
        *fail = 1;
        __hip_atomic_store(fail_word, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
  }
  __syncthreads();
}

// Q^{-1} of the leading n x n block of split_lds.ext (row major, identity
// outside the block), written back over it; with t != null the columns
// [col0, col0 + HC) also go to t (global, row major [NP][NP]).  The
// elimination is pipelined over the four waves (gj_inverse_pipe); its step
// records go to the rows of ext, which the waves have read by then.
__device__ __noinline__ void invert_split(int n, double2* t, int col0) {
  SplitLds& s = split_lds;
  constexpr int RB = NP / SW;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  double2 za[RB], zs[RB];
#pragma unroll
  for (int m = 0; m < RB; ++m) za[m] = s.ext[(RB * w + m) * NP + lane];
  const int pos = gj_inverse_pipe<SW>(za, zs, n, lane, w, s.ext, s.gj_piv, s.gj_pos, &s.gj_cnt, &s.flag_singular);
  const bool mine = t != nullptr && pos >= col0 && pos < col0 + HC;
#pragma unroll
  for (int m = 0; m < RB; ++m) {
    const int sl = RB * w + m;
    const int row = sl < n ? s.gj_piv[sl] : sl;
    const double2 val = sl < n ? zs[m] : make_double2(pos == sl ? 1.0 : 0.0, 0.0);
    s.ext[row * NP + pos] = val;
    if (mine) t[row * NP + pos] = val;
  }
  __syncthreads();
}

// D = [P_0 | P_1] T[:, col0 ..] for the wave's 16 x 32 block: P_h in pcx at
// h NP HC (row stride HC), T in tbuf (row stride NP).
template <class Epi>
__device__ __forceinline__ void split_gemm(const double2* __restrict__ pcx, const double2* __restrict__ tbuf, int lane,
                                           int RT, int col0, Epi&& epi) {
  __builtin_amdgcn_sched_barrier(0);
  d4 t1[NJT], t2[NJT], t3[NJT];
#pragma unroll
  for (int jt = 0; jt < NJT; ++jt) t1[jt] = t2[jt] = t3[jt] = d4{0, 0, 0, 0};
  const int ar = (16 * RT + (lane & 15)) * HC + (lane >> 4);
  const int bb = (lane >> 4) * NP + col0 + (lane & 15);
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const double2 u = q < 8 ? pcx[ar + 4 * q] : pcx[NP * HC + ar + 4 * (q - 8)];
    const double us = u.x + u.y;
#pragma unroll
    for (int jt = 0; jt < NJT; ++jt) {
      const double2 x = tbuf[bb + 4 * NP * q + 16 * jt];
      t1[jt] = mfma(u.x, x.x, t1[jt]);
      t2[jt] = mfma(u.y, x.y, t2[jt]);
      t3[jt] = mfma(us, x.x + x.y, t3[jt]);
    }
    if ((q & 3) == 3) __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int jt = 0; jt < NJT; ++jt)
#pragma unroll
    for (int v = 0; v < 4; ++v) epi(jt * 4 + v, t1[jt][v] - t2[jt][v], t3[jt][v] - t1[jt][v] - t2[jt][v]);
  __builtin_amdgcn_sched_barrier(0);
}

template <int SLOTS, int NT>
__device__ __forceinline__ void load_table_nodes(double2 (*tb)[MAXBOX + 1], const double2* __restrict__ Us, int box,
                                                 int n0, int n1, int tid) {
  const int total = (n1 - n0) * box;
  for (int e = tid; e < total; e += NT) {
    const int q = e / box;
    const int nn = n0 + q;
    tb[nn % SLOTS][e - q * box] = Us[(long long)nn * box + (e - q * box)];
  }
}

// Starts direct-to-LDS copies of nodes [n0, n1) of a structure's table into
// their ring slots: the (node, 64-entry chunk) pairs are dealt out over the
// SW waves, each chunk one 16-byte load per lane written at slot + 64 c + lane.
// The copies complete asynchronously; a wait for the vector memory counter
// followed by a workgroup barrier makes them visible.
template <int SLOTS>
__device__ __forceinline__ void prefetch_table_nodes(double2 (*tb)[MAXBOX + 1], const double2* __restrict__ Us,
                                                     int box, int n0, int n1, int w, int lane) {
  const int chunks = (box + 63) >> 6;
  const int total = (n1 - n0) * chunks;
  for (int t = __builtin_amdgcn_readfirstlane(w); t < total; t += SW) {
    const int q = t / chunks, c = t - q * chunks;
    const int nn = n0 + q;
    if (64 * c + lane < box)
      __builtin_amdgcn_global_load_lds((const void*)(Us + (long long)nn * box + 64 * c + lane),
                                       (__attribute__((address_space(3))) void*)(tb[nn % SLOTS] + 64 * c), 16, 0, 0);
  }
}

template <int STEPPER, bool BULK>
__global__ __launch_bounds__(ST, 1) void forward_split_kernel(FwdArgs a) {
  using T = Tab<STEPPER & 7>;
  SplitLds& s = split_lds;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int RT = w;                    // row tile of this wave
  const int pi = blockIdx.x >> 1, half = blockIdx.x & 1;  // launch slot of the pair, half
  const int p = a.pair_list ? a.pair_list[pi] : pi;
  if constexpr (BULK) {
    if (a.skip && a.skip[p]) return;   // both halves of the pair return here
  }
  const int col0 = HC * half;          // first column of this half
  const StructDev S = a.structs[a.pair_struct[p]];
  const int N = S.n_beams;
  const int L = S.n_slices;
  const double h = S.h;
  const double2* __restrict__ Us = a.U + S.table_off;

  if (tid < NP) {
    s.bhk[tid][0] = tid < N ? a.beams[2 * (S.beam_off + tid)] : 0;
    s.bhk[tid][1] = tid < N ? a.beams[2 * (S.beam_off + tid) + 1] : 0;
  }
  if (tid == 0) {
    s.flag_singular = 0;
    s.sync_fail = 0;
  }
  if (tid < T::slots) s.tb[tid][S.box] = make_double2(0.0, 0.0);
  __syncthreads();
  const double th0 = a.angles[2 * p], th1 = a.angles[2 * p + 1];
  if (tid < NP) {
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
  G2 gg;
#pragma unroll
  for (int v = 0; v < 4; ++v) gg.v[v] = s.g2s[16 * RT + 4 * v + (lane >> 4)];
  Gidx gx;
  {
    const int W = 2 * S.kd + 1;
    const int iA = 16 * RT + a_row<(STEPPER & F32_STAGES) != 0>(lane & 15);
    const int baseA = (s.bhk[iA][0] + S.hd) * W + (s.bhk[iA][1] + S.kd);
#pragma unroll
    for (int q = 0; q < 16; q += 2) {
      const int k0 = 4 * q + (lane >> 4), k1 = 4 * (q + 1) + (lane >> 4);
      const unsigned i0 = (iA < N && k0 < N) ? baseA - (s.bhk[k0][0] * W + s.bhk[k0][1]) : S.box;
      const unsigned i1 = (iA < N && k1 < N) ? baseA - (s.bhk[k1][0] * W + s.bhk[k1][1]) : S.box;
      gx.v[q >> 1] = i0 | (i1 << 16);
    }
  }
  double2* cb = s.cx;             // c of this half
  double2* xb = s.cx + NP * HC;   // stage input of this half
  int ob = (16 * RT + (lane >> 4)) * HC + (lane & 15);
  Mat d;
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const int row = 16 * RT + 4 * (e & 3) + (lane >> 4), col = col0 + 16 * (e >> 2) + (lane & 15);
    const bool dg = (row == col);
    cb[own<HC>(ob, e)] = make_double2(dg ? 1.0 : 0.0, 0.0);
    const double g2v = gg.v[e & 3];
    d.r[e] = (dg && g2v < 0.0) ? sqrt(-g2v) : 0.0;
    d.i[e] = (dg && g2v >= 0.0) ? sqrt(g2v) : 0.0;
    if constexpr (BULK) {
      if (row < N && col < N) {  // [I; Y] of a bulk below
        const double2 y = a.y_bottom[(long long)p * a.ld * a.ld + row * a.ld + col];
        d.r[e] = y.x;
        d.i[e] = y.y;
      }
    }
  }
  const bool save = a.ws != nullptr;
  char* pws = save ? a.ws + (long long)p * a.ck.pair_stride : nullptr;
  bool keep = save;  // as in forward_kernel
  if constexpr (BULK) keep = save && !a.final_only;
  char* X = a.xch + (long long)pi * XCH_STRIDE;
  unsigned long long* cnt_me = reinterpret_cast<unsigned long long*>(X) + half;
  unsigned long long* cnt_other = reinterpret_cast<unsigned long long*>(X) + (1 - half);
  double* xi_g = reinterpret_cast<double*>(X + XCH_XI);       // [half][parity][2][NP]
  double2* big_g = reinterpret_cast<double2*>(X + XCH_BIG);   // [half][parity][2][NP][HC]
  // launch number of this pair's block, kept in the block itself so that a
  // replayed launch (graph) moves on like a new one: both halves read it
  // here, half 0 writes it back after its last wait
  unsigned long long* ep_word = reinterpret_cast<unsigned long long*>(X) + 2;
  const unsigned long long epoch = __hip_atomic_load(ep_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
  // failure words of the two halves: the launch number in which the half gave up a wait
  unsigned long long* fail_me = reinterpret_cast<unsigned long long*>(X) + 3 + half;
  const unsigned long long* fail_other = reinterpret_cast<unsigned long long*>(X) + 3 + (1 - half);
  const bool give_up = a.xch_give_up == half;
  unsigned long long ev = epoch << 32;
  int nrhst = 0;
  // this half's [Q; P] columns to the exchange block of event ev
  auto publish_qp = [&]() {
    double2* mine = big_g + (long long)(half * 2 + (int)(ev & 1)) * 2 * NP * HC;
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int row = 16 * RT + 4 * (e & 3) + (lane >> 4), cl = 16 * (e >> 2) + (lane & 15);
      xput2(&mine[row * HC + cl], cb[own<HC>(ob, e)]);
      xput2(&mine[NP * HC + row * HC + cl], make_double2(d.r[e], d.i[e]));
    }
  };

  load_table_nodes<T::slots, ST>(s.tb, Us, S.box, 0, T::nodes + 1, tid);
  __syncthreads();
  for (int i = 0; i < L; ++i) {
    asm volatile("" : "+v"(ob));
    if (keep && (i % a.ck.every) == 0) {
      double2* st = reinterpret_cast<double2*>(pws + (long long)(i / a.ck.every) * a.ck.state_bytes);
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const int row = 16 * RT + 4 * (e & 3) + (lane >> 4), col = col0 + 16 * (e >> 2) + (lane & 15);
        st[row * NP + col] = cb[own<HC>(ob, e)];
        st[NP * NP + row * NP + col] = make_double2(d.r[e], d.i[e]);
      }
    }
    const int nb = i * T::nodes;
    d = rk_slice<STEPPER, HC>(cb, xb, &s.tb[0][0], nb, gx, gg, ob, lane, 0, h, d);
    // the next slice's new nodes go to the ring slots of this slice's first
    // nodes, which the last stage (node nb + nodes only) no longer reads
    if (i + 1 < L) prefetch_table_nodes<T::slots>(s.tb, Us, S.box, nb + T::nodes + 1, nb + 2 * T::nodes + 1, w, lane);

    // badness (Sec. 3.2): this half's row sums, then both halves' in half order
    {
      double dg[4] = {0, 0, 0, 0}, of[4] = {0, 0, 0, 0};
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const int row = 16 * RT + 4 * (e & 3) + (lane >> 4), col = col0 + 16 * (e >> 2) + (lane & 15);
        const double2 cv = cb[own<HC>(ob, e)];
        const double av = sqrt(cv.x * cv.x + cv.y * cv.y);
        if (row < N && col < N) {
          if (row == col) dg[e & 3] += av;
          else of[e & 3] += av;
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) {
          dg[v] += __shfl_xor(dg[v], off, 64);
          of[v] += __shfl_xor(of[v], off, 64);
        }
      }
      if ((lane & 15) == 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 16 * RT + 4 * v + (lane >> 4);
          s.xi_loc[0][row] = dg[v];
          s.xi_loc[1][row] = of[v];
        }
      }
    }
    __syncthreads();
    ++ev;
    if (tid < 2 * NP) xput(&xi_g[(half * 2 + (int)(ev & 1)) * 2 * NP + tid], s.xi_loc[tid / NP][tid % NP]);
    xch_publish(cnt_me, ev);
    xch_wait(cnt_other, ev, &s.sync_fail, fail_me, epoch, give_up);
    bool do_rhst;
    {
      const double* xo = xi_g + ((1 - half) * 2 + (int)(ev & 1)) * 2 * NP;
      const double dm = s.xi_loc[0][lane], om = s.xi_loc[1][lane], dt = xget(&xo[lane]), ot = xget(&xo[NP + lane]);
      const double dgl = half == 0 ? dm + dt : dt + dm;
      const double ofl = half == 0 ? om + ot : ot + om;
      double hi = lane < N ? dgl + ofl : 0.0;
      double lo = lane < N ? dgl - ofl : 1.0e308;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        hi = fmax(hi, __shfl_xor(hi, off, 64));
        lo = fmin(lo, __shfl_xor(lo, off, 64));
      }
      const double xi = lo > 0.0 ? hi / lo : INFINITY;
      do_rhst = xi > a.threshold;
    }
    if (keep && tid == 0 && half == 0) pws[a.ck.flags_off + i] = do_rhst ? 1 : 0;
    if (do_rhst) {
      // Z <- Z Q^{-1}: gather Q and P of both halves, invert Q, P <- P Q^{-1} for this half's columns
      ++nrhst;
      ++ev;
      publish_qp();
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const int row = 16 * RT + 4 * (e & 3) + (lane >> 4), cl = 16 * (e >> 2) + (lane & 15);
        s.ext[row * NP + col0 + cl] = cb[own<HC>(ob, e)];
      }
      __syncthreads();
      double2* pme = s.cx + half * NP * HC;   // P of half h goes to cx[h NP HC ..]
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const int row = 16 * RT + 4 * (e & 3) + (lane >> 4), cl = 16 * (e >> 2) + (lane & 15);
        pme[row * HC + cl] = make_double2(d.r[e], d.i[e]);
      }
      xch_publish(cnt_me, ev);
      xch_wait(cnt_other, ev, &s.sync_fail, fail_me, epoch, give_up);
      {
        // all of the partner's entries in flight at once, then into LDS
        const double2* theirs = big_g + (long long)((1 - half) * 2 + (int)(ev & 1)) * 2 * NP * HC;
        double2* pot = s.cx + (1 - half) * NP * HC;
        constexpr int PER = NP * HC / ST;
        double2 qv[PER], pv[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
          qv[q] = xget2(&theirs[tid + q * ST]);
          pv[q] = xget2(&theirs[NP * HC + tid + q * ST]);
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
          const int idx = tid + q * ST;
          const int r = idx / HC, c = idx - r * HC;
          s.ext[r * NP + HC * (1 - half) + c] = qv[q];
          pot[idx] = pv[q];
        }
      }
      __syncthreads();
      invert_split(N, keep ? reinterpret_cast<double2*>(pws + a.ck.q_off + (long long)i * NP * NP * sizeof(double2))
                           : nullptr,
                   col0);
      split_gemm(s.cx, s.ext, lane, RT, col0, [&](int e, double gr, double gi) {
        d.r[e] = gr;
        d.i[e] = gi;
      });
      if (keep && a.ck.r_off) {  // R = P Q^{-1} for an adjoint that keeps states only every few slices
        double2* rs = reinterpret_cast<double2*>(pws + a.ck.r_off + (long long)i * NP * NP * sizeof(double2));
#pragma unroll
        for (int e = 0; e < NE; ++e) {
          const int row = 16 * RT + 4 * (e & 3) + (lane >> 4), col = col0 + 16 * (e >> 2) + (lane & 15);
          rs[row * NP + col] = make_double2(d.r[e], d.i[e]);
        }
      }
      __syncthreads();
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const int row = 16 * RT + 4 * (e & 3) + (lane >> 4), col = col0 + 16 * (e >> 2) + (lane & 15);
        cb[own<HC>(ob, e)] = make_double2((row == col) ? 1.0 : 0.0, 0.0);
      }
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // table copies of the next slice
    __syncthreads();
  }

  if (save) {
    double2* st = reinterpret_cast<double2*>(pws + (long long)(a.ck.max_ckpt - 1) * a.ck.state_bytes);
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int row = 16 * RT + 4 * (e & 3) + (lane >> 4), col = col0 + 16 * (e >> 2) + (lane & 15);
      st[row * NP + col] = cb[own<HC>(ob, e)];
      st[NP * NP + row * NP + col] = make_double2(d.r[e], d.i[e]);
    }
  }
  // reflection (half 0): [Gamma Q - iP; Gamma Q + iP] of both halves, rho = lower (upper^{-1} e_1)
  ++ev;
  publish_qp();
  xch_publish(cnt_me, ev);
  if (half == 1) return;
  xch_wait(cnt_other, ev, &s.sync_fail, fail_me, epoch, give_up);
  if (tid == 0) {
    // the partner's failure word of this launch: released by its last counter raise, seen after the wait
    if (__hip_atomic_load(fail_other, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch) s.sync_fail = 1;
    __hip_atomic_store(ep_word, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  double2 low[NE];
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const int row = 16 * RT + 4 * (e & 3) + (lane >> 4), cl = 16 * (e >> 2) + (lane & 15);
    const double2 cv = cb[own<HC>(ob, e)];
    const double g2v = gg.v[e & 3];
    const double g_r = g2v >= 0.0 ? sqrt(g2v) : 0.0, g_i = g2v >= 0.0 ? 0.0 : -sqrt(-g2v);
    const double qr = g_r * cv.x - g_i * cv.y, qi = g_r * cv.y + g_i * cv.x;
    s.ext[row * NP + cl] = make_double2(qr + d.i[e], qi - d.r[e]);   // Gamma Q - iP
    low[e] = make_double2(qr - d.i[e], qi + d.r[e]);                  // Gamma Q + iP
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < NE; ++e) {
    const int row = 16 * RT + 4 * (e & 3) + (lane >> 4), cl = 16 * (e >> 2) + (lane & 15);
    s.cx[row * NP + cl] = low[e];
  }
  {
    const double2* theirs = big_g + (long long)(2 + (int)(ev & 1)) * 2 * NP * HC;
    for (int idx = tid; idx < NP * HC; idx += ST) {
      const int r = idx / HC, c = idx - r * HC;
      const double g2v = s.g2s[r];
      const double g_r = g2v >= 0.0 ? sqrt(g2v) : 0.0, g_i = g2v >= 0.0 ? 0.0 : -sqrt(-g2v);
      const double2 cv = xget2(&theirs[idx]), pv = xget2(&theirs[NP * HC + idx]);
      const double qr = g_r * cv.x - g_i * cv.y, qi = g_r * cv.y + g_i * cv.x;
      s.ext[r * NP + HC + c] = make_double2(qr + pv.y, qi - pv.x);
      s.cx[r * NP + HC + c] = make_double2(qr - pv.y, qi + pv.x);
    }
  }
  __syncthreads();
  // ||Gamma Q - iP||_inf for the breakdown test (as in forward_kernel)
  if (w == 0) {
    double rs = 0.0;
    if (lane < N)
      for (int k = 0; k < N; ++k) {
        const double2 v = s.ext[lane * NP + k];
        rs += sqrt(v.x * v.x + v.y * v.y);
      }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) rs = fmax(rs, __shfl_xor(rs, off, 64));
    if (lane == 0) s.bnorm = rs;
  }
  invert_split(N, nullptr, 0);
  if (tid < NP) {
    const int j = tid;
    double eta = 0.0;
    double2 rj = make_double2(0.0, 0.0);
    double xm = 0.0;
    if (j < N) {
      const double2 x = s.ext[j * NP];
      xm = sqrt(x.x * x.x + x.y * x.y);
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) xm = fmax(xm, __shfl_xor(xm, off, 64));
    const bool brk = !(s.bnorm * xm <= BREAKDOWN_COND);
    if (j < N) {
      for (int k = 0; k < N; ++k) {
        const double2 l = s.cx[j * NP + k], x = s.ext[k * NP];
        rj.x += l.x * x.x - l.y * x.y;
        rj.y += l.x * x.y + l.y * x.x;
      }
      const double g00 = s.g2s[0];
      const double gj = s.g2s[j];
      if (gj > 0.0) {
        eta = (rj.x * rj.x + rj.y * rj.y) * sqrt(g00) / sqrt(gj);
        if (a.convention == 1) eta *= sin(th0);
      }
    }
    const bool fin = isfinite(rj.x) && isfinite(rj.y);
    const unsigned long long bad = __ballot(!fin);
    int stv = 0;
    if (s.sync_fail) stv = 3;
    else if (s.flag_singular) stv = 1;
    else if (bad) stv = 2;
    else if (brk) stv = 4;
    if (stv != 0 && j < N) {  // a failed pair's outputs are NaN
      eta = NAN;
      rj = make_double2(NAN, NAN);
    }
    if (j < a.ld) {
      a.intensity[(long long)p * a.ld + j] = eta;
      if (a.rho) a.rho[(long long)p * a.ld + j] = rj;
    }
    for (int jt = NP + j; jt < a.ld; jt += NP) {  // outputs of a wider plan's padding
      a.intensity[(long long)p * a.ld + jt] = 0.0;
      if (a.rho) a.rho[(long long)p * a.ld + jt] = make_double2(0.0, 0.0);
    }
    if (j == 0) {
      a.status[p] = stv;
      if (a.nrhst) a.nrhst[p] = nrhst;
    }
  }
}

hipError_t launch_forward(int stepper, const FwdArgs& a, hipStream_t stream) {
  dim3 grid(a.n_pairs), block(FT);
  const bool bulk = a.y_bottom != nullptr;
  if ((stepper & 7) >= 2) {  // every splitting method; vacuum start only
    hipLaunchKernelGGL((forward_kernel<2, false>), grid, block, 0, stream, a);
  } else if (stepper == (0 | F32_STAGES)) {  // FP32 stage products; vacuum start only
    hipLaunchKernelGGL((forward_kernel<0 | F32_STAGES, false>), grid, block, 0, stream, a);
  } else if (stepper == (1 | F32_STAGES)) {
    hipLaunchKernelGGL((forward_kernel<1 | F32_STAGES, false>), grid, block, 0, stream, a);
  } else if (stepper == 0) {
    if (bulk)
      hipLaunchKernelGGL((forward_kernel<0, true>), grid, block, 0, stream, a);
    else
      hipLaunchKernelGGL((forward_kernel<0, false>), grid, block, 0, stream, a);
  } else {
    if (bulk)
      hipLaunchKernelGGL((forward_kernel<1, true>), grid, block, 0, stream, a);
    else
      hipLaunchKernelGGL((forward_kernel<1, false>), grid, block, 0, stream, a);
  }
  return hipGetLastError();
}

hipError_t launch_forward_split(int stepper, const FwdArgs& a, hipStream_t stream) {
  FwdArgs arg = a;
  void* params[] = {&arg};
  const bool bulk = a.y_bottom != nullptr;
  const void* f = stepper == (0 | F32_STAGES)   ? reinterpret_cast<const void*>(&forward_split_kernel<0 | F32_STAGES, false>)
                  : stepper == (1 | F32_STAGES) ? reinterpret_cast<const void*>(&forward_split_kernel<1 | F32_STAGES, false>)
                  : stepper == 0 ? (bulk ? reinterpret_cast<const void*>(&forward_split_kernel<0, true>)
                                         : reinterpret_cast<const void*>(&forward_split_kernel<0, false>))
                                 : (bulk ? reinterpret_cast<const void*>(&forward_split_kernel<1, true>)
                                         : reinterpret_cast<const void*>(&forward_split_kernel<1, false>));
  return hipLaunchCooperativeKernel(f, dim3(2 * a.n_pairs), dim3(ST), params, 0, stream);
}

int forward_split_max_pairs(int device) {
  int coop = 0, cus = 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) != hipSuccess || !coop) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  // the fewest resident workgroups per CU over every instantiation a split launch may use
  const void* fs[6] = {reinterpret_cast<const void*>(&forward_split_kernel<0, false>),
                       reinterpret_cast<const void*>(&forward_split_kernel<1, false>),
                       reinterpret_cast<const void*>(&forward_split_kernel<0, true>),
                       reinterpret_cast<const void*>(&forward_split_kernel<1, true>),
                       reinterpret_cast<const void*>(&forward_split_kernel<0 | F32_STAGES, false>),
                       reinterpret_cast<const void*>(&forward_split_kernel<1 | F32_STAGES, false>)};
  int per_cu = 1 << 30;
  for (const void* f : fs) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, ST, 0) != hipSuccess) return 0;
    per_cu = n < per_cu ? n : per_cu;
  }
  return cus * per_cu / 2;
}

}  // namespace rheed
