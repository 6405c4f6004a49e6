// Device helpers shared by the propagation kernels.
#pragma once
#include "rheed_internal.h"

namespace rheed {

// Wave-wide argmax of v (ties -> smaller index).
__device__ __forceinline__ void wave_argmax(double& v, int& idx) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double ov = __shfl_xor(v, off, 64);
    const int oi = __shfl_xor(idx, off, 64);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
}

// Column Gauss-Jordan with partial pivoting on Z = xb viewed as [128][64]:
// right-multiplies Z until its top block is I, so the bottom block becomes
// bottom * top^{-1}.  Only the leading n columns / pivots are processed.
// Each step copies the pivot column, column k and row k to LDS scratch, so
// that the update of every element reads only its own old value and copies.
__device__ __forceinline__ void gauss_jordan(double2* Z, double2* colp, double2* colk, double2* rowk, int* flag_singular,
                                             int n, int tid) {
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int j = lane;
  for (int k = 0; k < n; ++k) {
    const double2 zk = Z[k * NP + lane];
    double m2 = (lane >= k && lane < n) ? zk.x * zk.x + zk.y * zk.y : -1.0;
    int bi = lane;
    wave_argmax(m2, bi);
    if (!(m2 > 0.0) && tid == 0) *flag_singular = 1;
    if (tid < 2 * NP) {
      colp[tid] = Z[tid * NP + bi];
      colk[tid] = Z[tid * NP + k];
    } else if (tid < 3 * NP) {
      rowk[tid - 2 * NP] = Z[k * NP + (tid - 2 * NP)];
    }
    __syncthreads();
    if (j < n) {
      const double2 piv = rowk[bi];
      const double pn = piv.x * piv.x + piv.y * piv.y;
      const double2 ip = make_double2(piv.x / pn, -piv.y / pn);
      const double2 mj = rowk[j == bi ? k : j];
      const double2 f = make_double2(mj.x * ip.x - mj.y * ip.y, mj.x * ip.y + mj.y * ip.x);
      for (int m = 0; m < 2 * NP / NWAVES; ++m) {
        const int r = w + NWAVES * m;
        const double2 zp = colp[r];
        const double2 zo = (j == bi) ? colk[r] : Z[r * NP + j];
        double2 nv;
        if (j == k) {
          nv = make_double2(zp.x * ip.x - zp.y * ip.y, zp.x * ip.y + zp.y * ip.x);
        } else {
          nv = make_double2(zo.x - (f.x * zp.x - f.y * zp.y), zo.y - (f.x * zp.y + f.y * zp.x));
        }
        Z[r * NP + j] = nv;
      }
    }
    __syncthreads();
  }
}

}  // namespace rheed
