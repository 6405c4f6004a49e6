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

}  // namespace rheed
