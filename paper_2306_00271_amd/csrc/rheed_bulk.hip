// The bulk layer (Sec. 2.2, treatment of the bulk layer).
//
// Below the surface region the crystal continues as the ideal bulk, a stack
// of identical unit layers; the reflection matrix at the top of k layers
// converges as k grows, and the state the converged stack leaves at its top
// is the bottom condition of the surface.  The stack is propagated upward one
// unit layer per forward pass.  Between layers the state is carried in the
// normalised form [I; Y] that the right-hand-side transformation of
// Sec. 3.2 leaves (Y = P Q^{-1}), the vacuum below the stack being
// Y = i Gamma; the reflection matrix of the stack is
// R = (Gamma + iY)(Gamma - iY)^{-1} (the boundary matrix S applied to [I; Y],
// whose first column is rho(0) in Eq. vrhocomp).  bulk_update_kernel forms
// Y and R at the top of the layer every pair still iterating has just
// crossed, from the final state the forward pass kept in its workspace, and
// tests the change max_jk |R' - R| against the tolerance.
#include "rheed_internal.h"

namespace rheed {
namespace {

constexpr int BT = 256;  // threads of the one workgroup per pair
static_assert(BT % NP == 0, "each thread keeps one column in the elimination");

struct BulkLds {
  double2 m[2 * NP][NP + 1];  // [Q; P], then [Gamma - iY; Gamma + iY]; columns eliminated in place
  double2 f[NP];              // pivot row of the current step
  double g2s[NP];
  double red[BT / 64];
  int piv;
  int singular;
  int nonfinite;
};

__shared__ BulkLds bulk_lds;

__device__ inline double2 cmul(double2 x, double2 y) {
  return make_double2(x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x);
}

// Column Gauss-Jordan elimination with column pivoting on s.m = [B; A]
// (N x N blocks, B the identity outside its leading block): after N steps
// B is the identity and A holds A B^{-1} (column exchanges permute both
// blocks alike and cancel in the product).  Returns false for an exactly
// singular B.
__device__ bool eliminate(BulkLds& s, int N, int tid, int lane, int w) {
  for (int k = 0; k < N; ++k) {
    if (w == 0) {
      double v = -1.0;
      int ci = lane;
      if (lane >= k && lane < N) {
        const double2 x = s.m[k][lane];
        v = x.x * x.x + x.y * x.y;
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(v, off, 64);
        const int oc = __shfl_xor(ci, off, 64);
        if (ov > v || (ov == v && oc < ci)) {
          v = ov;
          ci = oc;
        }
      }
      if (lane == 0) {
        s.piv = ci;
        s.singular = !(v > 0.0);
      }
    }
    __syncthreads();
    if (s.singular) return false;  // uniform across the workgroup
    const int pc = s.piv;
    if (pc != k) {
      for (int r = tid; r < 2 * NP; r += BT) {
        const double2 t = s.m[r][k];
        s.m[r][k] = s.m[r][pc];
        s.m[r][pc] = t;
      }
      __syncthreads();
    }
    const double2 pv = s.m[k][k];
    const double den = pv.x * pv.x + pv.y * pv.y;
    const double2 inv = make_double2(pv.x / den, -pv.y / den);
    __syncthreads();
    for (int r = tid; r < 2 * NP; r += BT) s.m[r][k] = cmul(s.m[r][k], inv);
    __syncthreads();
    if (tid < NP) s.f[tid] = (tid != k && tid < N) ? s.m[k][tid] : make_double2(0.0, 0.0);
    __syncthreads();
    // column c -= f_c column k; each thread keeps one column (BT is a multiple
    // of 64) and its multiplier.  Rows N.. of each block are skipped: there
    // the eliminated columns hold 0 (identity rows of B, zero rows of A).
    {
      const int c = tid & (NP - 1);
      const double2 fc = s.f[c];
      if (fc.x != 0.0 || fc.y != 0.0) {
        for (int r = tid / NP; r < N; r += BT / NP) {
#pragma unroll
          for (int blk = 0; blk < 2; ++blk) {
            const double2 t = cmul(fc, s.m[blk * NP + r][k]);
            s.m[blk * NP + r][c].x -= t.x;
            s.m[blk * NP + r][c].y -= t.y;
          }
        }
      }
    }
    __syncthreads();
  }
  return true;
}

// Gamma^2 of pair p's beams into s.g2s (as in the forward pass).
__device__ void load_g2(BulkLds& s, const BulkArgs& a, const StructDev& S, int p, int tid) {
  if (tid < NP) {
    double arg = 0.0;
    if (tid < S.n_beams) {
      // Gamma_j^2 = gamma^2 - |b0 + k_j|^2, b0 = gamma cos(theta0) (cos theta1, sin theta1)
      const double th0 = a.angles[2 * p], th1 = a.angles[2 * p + 1];
      const int bh = a.beams[2 * (S.beam_off + tid)], bk = a.beams[2 * (S.beam_off + tid) + 1];
      const double qx = S.gamma * cos(th0) * cos(th1) + bh * S.recip[0] + bk * S.recip[2];
      const double qy = S.gamma * cos(th0) * sin(th1) + bh * S.recip[1] + bk * S.recip[3];
      arg = S.gamma * S.gamma - (qx * qx + qy * qy);
    }
    s.g2s[tid] = arg;
  }
}

__global__ __launch_bounds__(BT, 1) void bulk_update_kernel(BulkArgs a) {
  BulkLds& s = bulk_lds;
  const int p = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (a.done[p]) return;  // converged or failed at an earlier layer: Y and R stay
  if (a.fstatus[p] != 0) {  // this layer's forward pass failed: stop the pair with its status
    if (tid == 0) {
      a.status[p] = a.fstatus[p];
      a.done[p] = 1;
    }
    return;
  }
  const StructDev S = a.structs[a.pair_struct[p]];
  const int N = S.n_beams;
  const long long mbase = (long long)p * a.ld * a.ld;
  load_g2(s, a, S, p, tid);
  if (tid == 0) s.nonfinite = 0;
  // [Q; P] of the final state (row major [NP][NP] c, then c'), Q the identity
  // outside its leading N x N block
  const double2* st = reinterpret_cast<const double2*>(a.ws + (long long)p * a.ck.pair_stride +
                                                       (long long)(a.ck.max_ckpt - 1) * a.ck.state_bytes);
  for (int i = tid; i < NP * NP; i += BT) {
    const int j = i / NP, k = i - j * NP;
    const bool in = j < N && k < N;
    s.m[j][k] = in ? st[i] : make_double2(j == k ? 1.0 : 0.0, 0.0);
    s.m[NP + j][k] = in ? st[NP * NP + i] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  bool ok = eliminate(s, N, tid, lane, w);
  // this thread's entries i = tid + q BT of Y' and R', kept in registers until
  // the layer has passed (a pair that fails keeps its last Y and R)
  constexpr int PER = NP * NP / BT;
  double2 yv[PER], rv[PER];
  double dmax = 0.0;
  if (ok) {
    // Y' = P Q^{-1}, then [Gamma - iY'; Gamma + iY'] in place for R'
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int i = tid + q * BT, j = i / NP, k = i - j * NP;
      yv[q] = s.m[NP + j][k];
      double2 b = make_double2(j == k ? 1.0 : 0.0, 0.0), av = make_double2(0.0, 0.0);
      if (j < N && k < N) {
        if (!isfinite(yv[q].x) || !isfinite(yv[q].y)) s.nonfinite = 1;  // every writer stores 1
        const double2 g = j == k ? gamma_of(s.g2s[j]) : make_double2(0.0, 0.0);
        b = make_double2(g.x + yv[q].y, g.y - yv[q].x);    // Gamma - iY
        av = make_double2(g.x - yv[q].y, g.y + yv[q].x);   // Gamma + iY
      }
      s.m[j][k] = b;  // entry (j, k) is read and written by this thread only
      s.m[NP + j][k] = av;
    }
    __syncthreads();
    ok = eliminate(s, N, tid, lane, w);
  }
  if (ok) {
    // R' = (Gamma + iY')(Gamma - iY')^{-1}; the largest change against R
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int i = tid + q * BT, j = i / NP, k = i - j * NP;
      rv[q] = s.m[NP + j][k];
      if (j < N && k < N) {
        if (!isfinite(rv[q].x) || !isfinite(rv[q].y)) s.nonfinite = 1;
        const double2 o = a.r[mbase + (long long)j * a.ld + k];
        const double dx = rv[q].x - o.x, dy = rv[q].y - o.y;
        dmax = fmax(dmax, sqrt(dx * dx + dy * dy));
      }
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, off, 64));
  if (lane == 0) s.red[w] = dmax;
  __syncthreads();
  const bool fail = !ok || s.nonfinite;  // uniform: read after the barrier
  if (tid == 0) {
    double dm = s.red[0];
    for (int q = 1; q < BT / 64; ++q) dm = fmax(dm, s.red[q]);
    if (fail) {
      a.status[p] = ok ? 2 : 1;  // RHEED_PAIR_NONFINITE : RHEED_PAIR_SINGULAR
      a.done[p] = 1;
    } else if (dm <= a.tol) {
      a.done[p] = 1;
      a.layers[p] = a.iter;
    }
  }
  if (fail) return;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int i = tid + q * BT, j = i / NP, k = i - j * NP;
    if (j < N && k < N) {
      a.y[mbase + (long long)j * a.ld + k] = yv[q];
      a.r[mbase + (long long)j * a.ld + k] = rv[q];
    }
  }
}

// The vacuum below the stack: Y = i Gamma (diagonal), R = 0; flags cleared.
__global__ __launch_bounds__(BT, 1) void bulk_init_kernel(BulkArgs a) {
  BulkLds& s = bulk_lds;
  const int p = blockIdx.x, tid = threadIdx.x;
  const StructDev S = a.structs[a.pair_struct[p]];
  load_g2(s, a, S, p, tid);
  __syncthreads();
  const long long mbase = (long long)p * a.ld * a.ld;
  for (int i = tid; i < a.ld * a.ld; i += BT) {
    const int j = i / a.ld, k = i - j * a.ld;
    double2 y = make_double2(0.0, 0.0);
    if (j == k && j < S.n_beams) {
      const double g2 = s.g2s[j];
      y = make_double2(g2 < 0.0 ? sqrt(-g2) : 0.0, g2 >= 0.0 ? sqrt(g2) : 0.0);  // i Gamma_j
    }
    a.y[mbase + i] = y;
    a.r[mbase + i] = make_double2(0.0, 0.0);
  }
  if (tid == 0) {
    a.done[p] = 0;
    a.layers[p] = -1;
    a.status[p] = 0;
  }
}

}  // namespace

hipError_t launch_bulk_update(const BulkArgs& a, hipStream_t stream) {
  hipLaunchKernelGGL(bulk_update_kernel, dim3(a.n_pairs), dim3(BT), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_bulk_init(const BulkArgs& a, hipStream_t stream) {
  hipLaunchKernelGGL(bulk_init_kernel, dim3(a.n_pairs), dim3(BT), 0, stream, a);
  return hipGetLastError();
}

}  // namespace rheed
