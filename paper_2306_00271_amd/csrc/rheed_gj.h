// Device helpers shared by the propagation kernels.
#pragma once
#include "rheed_internal.h"

namespace rheed {

// Maximum of a 32-bit key over the wave by DPP: butterflies inside rows of 16
// lanes, then the row broadcasts; the result is read from lane 63.
#define RHEED_DPP_MAX_STEP(CTRL, RMASK)                                                    \
  {                                                                                        \
    const unsigned o = (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, CTRL, RMASK, 0xf, false); \
    v = o > v ? o : v;                                                                     \
  }
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  RHEED_DPP_MAX_STEP(0xB1, 0xf)   // quad_perm [1,0,3,2]
  RHEED_DPP_MAX_STEP(0x4E, 0xf)   // quad_perm [2,3,0,1]
  RHEED_DPP_MAX_STEP(0x141, 0xf)  // row_half_mirror
  RHEED_DPP_MAX_STEP(0x140, 0xf)  // row_mirror
  RHEED_DPP_MAX_STEP(0x142, 0xa)  // row_bcast:15
  RHEED_DPP_MAX_STEP(0x143, 0xc)  // row_bcast:31
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}
#undef RHEED_DPP_MAX_STEP

// Value of v in lane l (wave-uniform l), through scalar registers.
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Register-resident inversion by column Gauss-Jordan elimination with partial
// pivoting and no column exchanges.  A workgroup of NWV waves holds the n x n
// matrix A (padded to NP x NP) column-wise: lane j of wave w keeps column j of
// rows w + NWV m of A in z[m], m < IB = NP / NWV.  Step k picks, among the
// columns not yet used, the one with the largest |A_kj| (pc_k), scales it so
// that A_{k,pc_k} = 1 and subtracts it from every other column so that row k
// becomes a unit row.  The same column operations, applied to I, give A^{-1};
// row pc_k of that product is untouched (e_{pc_k}^T) until step k, so it is
// kept in slot k only from step k on: slot s = w + NWV (m - IB) lives in z[m],
// m >= IB.  At the end slot s < n holds row pc_s of A^{-1}, with the entry of
// column c of A^{-1} in the lane whose column was the pivot of step c (the
// returned position; columns >= n keep their own, and their rows < n of A must
// be zero, as padding is).  pivrec[s] = pc_s.  Per step every wave updates
// about IB + 1 rows per lane: the rows k.. of A and the slots ..k.
// Per step: one workgroup barrier.  Row k, written to LDS by the wave that
// owns it as soon as the previous step has produced it, is read by every
// wave, which finds the pivot itself: the key of column j is the upper 32 bits
// of the bit pattern of |A_kj|^2 (sign, exponent and 20 mantissa bits, so
// candidates within a relative 2^-14 count as equal) with the low 6 bits
// replaced by 63 - j (ties go to the smaller index), reduced by DPP.  Rows of
// A above row k and slots not yet in use are updated too: their entries in
// the pivot column are zero, so they do not change.  The pivot column reaches
// the other lanes of a wave through scalar registers (v_readlane).
//   rowbuf: 2 NP entries, pivrec: NP ints.
template <int NWV, int KB>
struct GjInv {
  static constexpr int IB = NP / NWV, RM = 2 * NP / NWV;
  static __device__ __forceinline__ void run(double2 (&z)[RM], int n, int lane, int wu, bool& used, int& pos,
                                             double2* rowbuf, int* pivrec, int* flag_singular) {
    if (KB * NWV >= n) return;
    // not unrolled: the straight-line code of all steps would not stay in
    // the instruction cache, and each step runs once per elimination
#pragma unroll 1
    for (int kk = 0; kk < NWV; ++kk) {
      const int k = KB * NWV + kk;
      if (k >= n) return;
      const int slot = k & 1;
      __syncthreads();
      const double2 v = rowbuf[slot * NP + lane];
      const double m2 = v.x * v.x + v.y * v.y;
      unsigned key = 0;
      if (!used && lane < n)
        key = ((unsigned)(((unsigned long long)__double_as_longlong(m2)) >> 32) & ~63u) | (unsigned)(63 - lane);
      key = wave_max_u32(key);
      if ((key >> 6) == 0 && lane == 0 && wu == 0) *flag_singular = 1;
      const int pc = 63 - (int)(key & 63);
      if (lane == 0 && wu == 0) pivrec[k] = pc;
      if (wu == kk) z[IB + KB] = make_double2(lane == pc ? 1.0 : 0.0, 0.0);  // slot k starts as e_pc
      if (lane == pc) {
        used = true;
        pos = k;
      }
      // the pivot column of this wave's rows, from lane pc through scalar registers
      double2 zp[RM];
#pragma unroll
      for (int m = KB; m <= IB + KB; ++m) zp[m] = make_double2(readlane_f64(z[m].x, pc), readlane_f64(z[m].y, pc));
      const double2 piv = make_double2(readlane_f64(v.x, pc), readlane_f64(v.y, pc));
      const double inv = 1.0 / (piv.x * piv.x + piv.y * piv.y);
      const double2 ip = make_double2(piv.x * inv, -piv.y * inv);
      // column pc becomes z ip = z - (1 - ip) z; every other column z - (a_kj ip) z_pc
      double2 f = make_double2(v.x * ip.x - v.y * ip.y, v.x * ip.y + v.y * ip.x);
      if (lane == pc) f = make_double2(1.0 - ip.x, -ip.y);
#pragma unroll
      for (int m = KB; m <= IB + KB; ++m) {
        z[m].x = fma(-f.x, zp[m].x, z[m].x);
        z[m].x = fma(f.y, zp[m].y, z[m].x);
        z[m].y = fma(-f.x, zp[m].y, z[m].y);
        z[m].y = fma(-f.y, zp[m].x, z[m].y);
      }
      // publish row k + 1 (owned by wave (k + 1) % NWV, register (k + 1) / NWV)
      if (k + 1 < n && wu == (k + 1) % NWV) {
        const double2 rv = ((k + 1) / NWV == KB) ? z[KB] : z[KB + 1 < IB ? KB + 1 : KB];
        rowbuf[(slot ^ 1) * NP + lane] = rv;
      }
    }
    GjInv<NWV, KB + 1>::run(z, n, lane, wu, used, pos, rowbuf, pivrec, flag_singular);
  }
};

template <int NWV>
struct GjInv<NWV, NP / NWV> {
  static __device__ __forceinline__ void run(double2 (&)[2 * NP / NWV], int, int, int, bool&, int&, double2*, int*,
                                             int*) {}
};

// z[m < NP / NWV]: rows of A as above; z[m >= NP / NWV] is overwritten.
// Returns this lane's column position; pivrec is valid after the call.
template <int NWV>
__device__ __forceinline__ int gj_inverse(double2 (&z)[2 * NP / NWV], int n, int lane, int w, double2* rowbuf,
                                          int* pivrec, int* flag_singular) {
  bool used = false;
  int pos = lane;
  const int wu = __builtin_amdgcn_readfirstlane(w);
#pragma unroll
  for (int m = NP / NWV; m < 2 * NP / NWV; ++m) z[m] = make_double2(0.0, 0.0);
  if (wu == 0) rowbuf[lane] = z[0];  // row 0
  GjInv<NWV, 0>::run(z, n, lane, wu, used, pos, rowbuf, pivrec, flag_singular);
  __syncthreads();
  return pos;
}

// The same elimination as a pipeline over the waves, for a workgroup of NWV
// waves on NWV SIMDs (the arithmetic of every step is that of GjInv, so the
// result is the same bit for bit).  Wave w holds rows RB w .. RB w + RB - 1
// of A (RB = NP / NWV) in za.  Step k is taken by the wave that owns row k,
// alone and without a workgroup barrier: row k is in its registers with every
// earlier step applied, so it picks the pivot, writes the step's multipliers
// f to rec[k][.] and pc_k to pivrec[k], raises the step counter (a
// workgroup-scope release store in LDS) and applies the step to its later
// rows.  The other waves apply the published steps in order: to their rows
// of A before their own block, and to the inverse rows of their block (zs)
// after it.  Inverse row pc_s is e_{pc_s} until step s (earlier steps leave
// it unchanged: its entry in their pivot columns is zero), so once the
// block's steps are recorded its inverse rows are formed from them and take
// the later blocks' steps as these come.
// A wave waits only for the step it applies next, and every step depends on
// earlier steps alone, so every wait ends.  A wait that finds the matrix
// already flagged singular returns at once (the results are discarded then),
// and one that still exceeds GJ_PIPE_SPIN polls flags it and gives up, so no
// wave can spin for long whatever the data.  rec may be the
// matrix's own storage (row k of it is read only by the wave that owns row
// k, before step k); posrec[j] ends as the step at which column j was the
// pivot (j if none).  Returns this lane's position, as gj_inverse.
constexpr int GJ_PIPE_SPIN = 1 << 18;

// Waits until more than k steps are published; returns the count it saw
// (k + 1 if the wait gave up).
__device__ __forceinline__ int gj_wait_step(const int* cnt, int k, int* flag_singular) {
  int it = 0;
  for (;;) {
    const int c =
        __builtin_amdgcn_readfirstlane(__hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
    if (c > k) return c;
    if (__builtin_amdgcn_readfirstlane(
            __hip_atomic_load(flag_singular, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) != 0 ||
        ++it > GJ_PIPE_SPIN) {
      *flag_singular = 1;
      return k + 1;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// Step (pc, f) on rows M0 .. M1 - 1 of z: z_m <- z_m - f z_m[pc].
template <int RB, int M0, int M1 = RB>
__device__ __forceinline__ void gj_apply(double2 (&z)[RB], int pc, double2 f) {
  double2 zp[RB];
#pragma unroll
  for (int m = M0; m < M1; ++m) zp[m] = make_double2(readlane_f64(z[m].x, pc), readlane_f64(z[m].y, pc));
#pragma unroll
  for (int m = M0; m < M1; ++m) {
    z[m].x = fma(-f.x, zp[m].x, z[m].x);
    z[m].x = fma(f.y, zp[m].y, z[m].x);
    z[m].y = fma(-f.x, zp[m].y, z[m].y);
    z[m].y = fma(-f.y, zp[m].x, z[m].y);
  }
}

// Published steps kb .. ke - 1 on all rows of z, in order.  avail counts the
// steps known to be published (from the last look at the counter); the next
// step's record is read while the current one is applied whenever it is
// known to be there, and the counter is looked at again only when avail runs
// out.  With USED, the pivot columns are collected in *um.
template <int RB, bool USED>
__device__ __forceinline__ void gj_consume(double2 (&z)[RB], int kb, int ke, int lane, int& avail,
                                           unsigned long long* um, const double2* rec, const int* pivrec,
                                           const int* cnt, int* flag_singular) {
  if (kb >= ke) return;
  if (kb >= avail) avail = gj_wait_step(cnt, kb, flag_singular);
  double2 f = rec[kb * NP + lane];
  int pv = pivrec[kb];
#pragma unroll 1
  for (int k = kb; k < ke; ++k) {
    const int pc = __builtin_amdgcn_readfirstlane(pv) & 63;
    const int k1 = k + 1;
    if (k1 < ke && k1 >= avail)  // a look without waiting
      avail = __builtin_amdgcn_readfirstlane(__hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
    const bool ahead = k1 < ke && k1 < avail;
    double2 fn = f;
    int pn = pv;
    if (ahead) {
      fn = rec[k1 * NP + lane];
      pn = pivrec[k1];
    }
    if (USED) *um |= 1ull << pc;
    gj_apply<RB, 0>(z, pc, f);
    if (k1 < ke && !ahead) {
      avail = gj_wait_step(cnt, k1, flag_singular);
      fn = rec[k1 * NP + lane];
      pn = pivrec[k1];
    }
    f = fn;
    pv = pn;
  }
}

// A wave's own block of steps, step by step (used for the block that
// reaches the matrix's last row; full blocks run as GjPanelPipe below).  The
// singular test accumulates in sing.
template <int NWV, int J>
struct GjPanel {
  static constexpr int RB = NP / NWV;
  static constexpr int J2 = J + 2 < RB ? J + 2 : RB;
  static __device__ __forceinline__ void run(double2 (&za)[RB], int n, int lane, int k0, unsigned long long& um,
                                             bool& sing, double2* rec, int* pivrec, int* posrec, int* cnt) {
    const int k = k0 + J;
    if (k >= n) return;
    const double2 v = za[J];
    const double m2 = v.x * v.x + v.y * v.y;
    unsigned key = 0;
    if (!((um >> lane) & 1ull) && lane < n)
      key = ((unsigned)(((unsigned long long)__double_as_longlong(m2)) >> 32) & ~63u) | (unsigned)(63 - lane);
    key = wave_max_u32(key);
    sing |= (key >> 6) == 0;
    const int pc = 63 - (int)(key & 63);
    um |= 1ull << pc;
    const double2 piv = make_double2(readlane_f64(v.x, pc), readlane_f64(v.y, pc));
    const double inv = 1.0 / (piv.x * piv.x + piv.y * piv.y);
    const double2 ip = make_double2(piv.x * inv, -piv.y * inv);
    double2 f = make_double2(v.x * ip.x - v.y * ip.y, v.x * ip.y + v.y * ip.x);
    if (lane == pc) f = make_double2(1.0 - ip.x, -ip.y);
    rec[k * NP + lane] = f;
    pivrec[k] = pc;  // every lane stores the same value
    posrec[pc] = k;
    gj_apply<RB, J + 1, J2>(za, pc, f);  // row k itself is not used again
    __hip_atomic_store(cnt, k + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    gj_apply<RB, J2, RB>(za, pc, f);
    GjPanel<NWV, J + 1>::run(za, n, lane, k0, um, sing, rec, pivrec, posrec, cnt);
  }
};
template <int NWV>
struct GjPanel<NWV, NP / NWV> {
  static __device__ __forceinline__ void run(double2 (&)[NP / NWV], int, int, int, unsigned long long&, bool&,
                                             double2*, int*, int*, int*) {}
};

// The full block as a software pipeline: step J's pivot search, division
// and multipliers run in eight pieces (key, the six DPP stages, the pivot
// and its reciprocal), and step J - 1's update of rows J + 1 .. RB - 1,
// deferred to here, is cut into eight chunks placed after the pieces, with
// scheduling barriers between them, so that the row updates fill the latency
// of the search.  Row J + 1 takes step J - 1 in the first chunk that holds
// it and step J right after the multipliers are known, so every row still
// takes its steps in order, with the same arithmetic.
template <int RB, int D0, int ND, int I>
__device__ __forceinline__ void gj_chunk(double2 (&za)[RB], int pc, double2 f) {
  if constexpr (ND > 0) gj_apply<RB, D0 + ND * I / 8, D0 + ND * (I + 1) / 8>(za, pc, f);
  __builtin_amdgcn_sched_barrier(0);
}

template <int NWV, int J>
struct GjPanelPipe {
  static constexpr int RB = NP / NWV;
  static constexpr int D0 = J + 1, ND = J == 0 ? 0 : RB - (J + 1);  // rows waiting for step J - 1
  static __device__ __forceinline__ void run(double2 (&za)[RB], int n, int lane, int k0, unsigned long long& um,
                                             bool& sing, double2* rec, int* pivrec, int* posrec, int* cnt, int pcp,
                                             double2 fp) {
    const int k = k0 + J;
    const double2 v = za[J];
    const double m2 = v.x * v.x + v.y * v.y;
    unsigned key = 0;
    if (!((um >> lane) & 1ull) && lane < n)
      key = ((unsigned)(((unsigned long long)__double_as_longlong(m2)) >> 32) & ~63u) | (unsigned)(63 - lane);
    gj_chunk<RB, D0, ND, 0>(za, pcp, fp);
    unsigned o = (unsigned)__builtin_amdgcn_update_dpp((int)key, (int)key, 0xB1, 0xf, 0xf, false);
    key = o > key ? o : key;
    gj_chunk<RB, D0, ND, 1>(za, pcp, fp);
    o = (unsigned)__builtin_amdgcn_update_dpp((int)key, (int)key, 0x4E, 0xf, 0xf, false);
    key = o > key ? o : key;
    gj_chunk<RB, D0, ND, 2>(za, pcp, fp);
    o = (unsigned)__builtin_amdgcn_update_dpp((int)key, (int)key, 0x141, 0xf, 0xf, false);
    key = o > key ? o : key;
    gj_chunk<RB, D0, ND, 3>(za, pcp, fp);
    o = (unsigned)__builtin_amdgcn_update_dpp((int)key, (int)key, 0x140, 0xf, 0xf, false);
    key = o > key ? o : key;
    gj_chunk<RB, D0, ND, 4>(za, pcp, fp);
    o = (unsigned)__builtin_amdgcn_update_dpp((int)key, (int)key, 0x142, 0xa, 0xf, false);
    key = o > key ? o : key;
    gj_chunk<RB, D0, ND, 5>(za, pcp, fp);
    o = (unsigned)__builtin_amdgcn_update_dpp((int)key, (int)key, 0x143, 0xc, 0xf, false);
    key = o > key ? o : key;
    key = (unsigned)__builtin_amdgcn_readlane((int)key, 63);
    sing |= (key >> 6) == 0;
    const int pc = 63 - (int)(key & 63);
    um |= 1ull << pc;
    const double2 piv = make_double2(readlane_f64(v.x, pc), readlane_f64(v.y, pc));
    gj_chunk<RB, D0, ND, 6>(za, pcp, fp);
    const double inv = 1.0 / (piv.x * piv.x + piv.y * piv.y);
    const double2 ip = make_double2(piv.x * inv, -piv.y * inv);
    double2 f = make_double2(v.x * ip.x - v.y * ip.y, v.x * ip.y + v.y * ip.x);
    if (lane == pc) f = make_double2(1.0 - ip.x, -ip.y);
    gj_chunk<RB, D0, ND, 7>(za, pcp, fp);
    rec[k * NP + lane] = f;
    pivrec[k] = pc;  // every lane stores the same value
    posrec[pc] = k;
    if constexpr (J + 1 < RB) gj_apply<RB, J + 1, J + 2>(za, pc, f);
    __hip_atomic_store(cnt, k + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    GjPanelPipe<NWV, J + 1>::run(za, n, lane, k0, um, sing, rec, pivrec, posrec, cnt, pc, f);
  }
};
template <int NWV>
struct GjPanelPipe<NWV, NP / NWV> {
  static __device__ __forceinline__ void run(double2 (&)[NP / NWV], int, int, int, unsigned long long&, bool&,
                                             double2*, int*, int*, int*, int, double2) {}
};

// The inverse rows of a wave's own block through its own steps: row J is
// e_{pc} before step k0 + J, which it then takes with rows 0 .. J - 1.
template <int RB, int J>
struct GjOwnRows {
  static __device__ __forceinline__ void run(double2 (&zs)[RB], int n, int lane, int k0, const double2* rec,
                                             const int* pivrec) {
    const int k = k0 + J;
    if (k >= n) return;
    const double2 f = rec[k * NP + lane];
    const int pc = __builtin_amdgcn_readfirstlane(pivrec[k]) & 63;
    zs[J] = make_double2(lane == pc ? 1.0 : 0.0, 0.0);
    gj_apply<RB, 0, J + 1>(zs, pc, f);
    GjOwnRows<RB, J + 1>::run(zs, n, lane, k0, rec, pivrec);
  }
};
template <int RB>
struct GjOwnRows<RB, RB> {
  static __device__ __forceinline__ void run(double2 (&)[RB], int, int, int, const double2*, const int*) {}
};

//   za: rows of A as above (rows >= n must be those of the identity);
//   zs: out, inverse row pivrec[RB w + m] in zs[m] for RB w + m < n.
//   rec: n x NP entries; pivrec, posrec: NP ints; cnt: one int.
template <int NWV>
__device__ __forceinline__ int gj_inverse_pipe(double2 (&za)[NP / NWV], double2 (&zs)[NP / NWV], int n, int lane,
                                               int w, double2* rec, int* pivrec, int* posrec, int* cnt,
                                               int* flag_singular) {
  constexpr int RB = NP / NWV;
  const int wu = __builtin_amdgcn_readfirstlane(w);
  const int k0 = RB * wu;
  if (wu == 0) {
    posrec[lane] = lane;
    if (lane == 0) *cnt = 0;
  }
#pragma unroll
  for (int m = 0; m < RB; ++m) zs[m] = make_double2(0.0, 0.0);
  __syncthreads();
  if (k0 < n) {
    unsigned long long um = 0;
    int avail = 0;
    gj_consume<RB, true>(za, 0, k0, lane, avail, &um, rec, pivrec, cnt, flag_singular);  // earlier blocks' steps
    bool sing = false;
    if (k0 + RB <= n)
      GjPanelPipe<NWV, 0>::run(za, n, lane, k0, um, sing, rec, pivrec, posrec, cnt, 0, make_double2(0.0, 0.0));
    else
      GjPanel<NWV, 0>::run(za, n, lane, k0, um, sing, rec, pivrec, posrec, cnt);
    if (sing && lane == 0) *flag_singular = 1;
    GjOwnRows<RB, 0>::run(zs, n, lane, k0, rec, pivrec);
    gj_consume<RB, false>(zs, k0 + RB, n, lane, avail, nullptr, rec, pivrec, cnt, flag_singular);
  }
  __syncthreads();
  return posrec[lane];
}

}  // namespace rheed
