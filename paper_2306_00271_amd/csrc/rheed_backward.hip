// Adjoint of the forward propagation (not in the paper), on gfx950.
//
// Only the first column of the reflection matrix is used (rho(0) = R e_1,
// Algorithm 1), so the cotangent of every intermediate state is rank one:
// if the final state Z_L has cotangent y x^H, then
//   * through a slice map Z <- Phi Z (an RK step is linear from the left)
//     the cotangent becomes (Phi^H y) x^H;
//   * through a right-hand-side transformation Z' = Z Q^{-1} (Sec. 3.2) it
//     becomes y x^H with x = Q^{-1} x' and y = y' - [Z'^H y'; 0]; the second
//     term is the derivative of Q^{-1} itself.  The output is invariant under
//     right multiplication of Z, so in exact arithmetic that term changes
//     nothing, but it removes the components of y that the backward
//     recursion would amplify;
//   * the gradient of the coupling matrix at stage r is g_r v_r^H with v_r the
//     stage input of the RK step applied to the single physical column
//     psi = Z x, and g_r the adjoint of that stage's product.
// One workgroup per (structure, angle) pair therefore walks the slices
// backwards with vectors only: x is carried back through the stored upper
// blocks Q (x <- Q^{-1} x where a transformation happened), psi = Z_i x comes
// from the stored slice-start states, and each stage costs a few N x N
// matrix-vector products.  Gradients land in a per-pair table of rod
// differences; a second kernel sums them over the angles of each structure
// in a fixed order.
//
// Final step (Eq. vrhocomp, first column): with B = Gamma Q - iP,
// A = Gamma Q + iP, B x = e_1, rho = A x and
// eta_j = w_j |rho_j|^2 (w_j = Gamma_0/Gamma_j on open beams, times sin theta0
// in the printed normalisation):
//   rho_bar_j = 2 w_j rho_j dL/deta_j,  x_bar = A^H rho_bar,  w = B^{-H} x_bar,
//   cotangent of Z_L = [conj(Gamma)(rho_bar - w); -i (rho_bar + w)] x^H.
#include "rheed_internal.h"
#include "rheed_gj.h"

namespace rheed {

struct StageVecs {
  double2 yc[7][NP], yd[7][NP];    // stage inputs of the RK step applied to psi
  double2 kd[7][NP];               // K^(c') of each stage
  double2 ybc[7][NP], ybd[7][NP];  // stage-input cotangents
};

struct BLds {
  union {
    double2 zb[2 * NP * NP];   // elimination workspace [top; bottom]
    StageVecs sv;              // per-slice vectors (the eliminations of a slice finish before its stages start)
  };
  double2 tb[1][MAXBOX + 1];   // node table of the current stage; entry box = 0
  double2 gj_colp[2 * NP];
  double2 gj_colk[2 * NP];
  double2 gj_rowk[NP];
  double2 x[NP];               // coefficients of the physical column
  double2 pc[NP], pd[NP];      // psi = Z x: c and c' parts
  double2 cb_[NP], db_[NP];    // running cotangent y = (c_bar, c'_bar)
  double2 tmp[NP], tmp2[NP];
  double g2s[NP];
  int bhk[NP][2];
  int offk[NP];                // h_k W + k_k
  int basej[NP];               // (h_j + Hd) W + k_j + Kd
  int flag_singular;
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// out = M v (herm = false) or M^H v (herm = true) with M = U(node) + Gamma^2,
// U_{jk} = table[idx(j, k)]; 4 threads per row, rows < n.
__device__ __forceinline__ void matvec_u(BLds& s, const double2* tslot, const double2* v, double2* out, bool herm,
                                         int n, int box, int tid) {
  const int j = tid >> 2, part = tid & 3;
  double2 acc = make_double2(0.0, 0.0);
  if (j < n) {
    for (int k = part; k < n; k += 4) {
      const int idx = herm ? (s.basej[k] - s.offk[j]) : (s.basej[j] - s.offk[k]);
      const double2 u = tslot[idx];
      acc = herm ? make_double2(acc.x + u.x * v[k].x + u.y * v[k].y, acc.y + u.x * v[k].y - u.y * v[k].x)
                 : make_double2(acc.x + u.x * v[k].x - u.y * v[k].y, acc.y + u.x * v[k].y + u.y * v[k].x);
    }
  }
  acc.x += __shfl_xor(acc.x, 1, 64);
  acc.y += __shfl_xor(acc.y, 1, 64);
  acc.x += __shfl_xor(acc.x, 2, 64);
  acc.y += __shfl_xor(acc.y, 2, 64);
  if (part == 0 && j < NP) {
    if (j < n) out[j] = make_double2(acc.x + s.g2s[j] * v[j].x, acc.y + s.g2s[j] * v[j].y);
    else out[j] = make_double2(0.0, 0.0);
  }
  (void)box;
}

// out = Mat v for a dense [NP][NP] complex matrix in global memory (rows < n)
__device__ __forceinline__ void matvec_dense(const double2* __restrict__ Mg, const double2* v, double2* out, int n,
                                             int tid) {
  const int j = tid >> 2, part = tid & 3;
  double2 acc = make_double2(0.0, 0.0);
  if (j < n)
    for (int k = part; k < n; k += 4) {
      const double2 m = Mg[j * NP + k];
      acc.x += m.x * v[k].x - m.y * v[k].y;
      acc.y += m.x * v[k].y + m.y * v[k].x;
    }
  acc.x += __shfl_xor(acc.x, 1, 64);
  acc.y += __shfl_xor(acc.y, 1, 64);
  acc.x += __shfl_xor(acc.x, 2, 64);
  acc.y += __shfl_xor(acc.y, 2, 64);
  if (part == 0 && j < NP) out[j] = j < n ? acc : make_double2(0.0, 0.0);
}

// out = Mat^H v for a dense [NP][NP] complex matrix in global memory (n x n)
__device__ __forceinline__ void matvec_dense_h(const double2* __restrict__ Mg, const double2* v, double2* out, int n,
                                               int tid) {
  const int k = tid >> 2, part = tid & 3;
  double2 acc = make_double2(0.0, 0.0);
  if (k < n)
    for (int j = part; j < n; j += 4) {
      const double2 m = Mg[j * NP + k];
      acc.x += m.x * v[j].x + m.y * v[j].y;
      acc.y += m.x * v[j].y - m.y * v[j].x;
    }
  acc.x += __shfl_xor(acc.x, 1, 64);
  acc.y += __shfl_xor(acc.y, 1, 64);
  acc.x += __shfl_xor(acc.x, 2, 64);
  acc.y += __shfl_xor(acc.y, 2, 64);
  if (part == 0 && k < NP) out[k] = k < n ? acc : make_double2(0.0, 0.0);
}

// Loads M (global, [NP][NP]) into the top block and I into the bottom block,
// eliminates, and leaves M^{-1} (leading n x n) in the bottom block.
__device__ __forceinline__ void invert_into_bottom(BLds& s, const double2* __restrict__ Mg, int n, int tid) {
  for (int e = tid; e < NP * NP; e += NTHREADS) {
    const int r = e / NP, c = e - r * NP;
    s.zb[e] = (r < n && c < n) ? Mg[e] : make_double2(r == c ? 1.0 : 0.0, 0.0);
    s.zb[NP * NP + e] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  gauss_jordan(s.zb, s.gj_colp, s.gj_colk, s.gj_rowk, &s.flag_singular, n, tid);
}

__device__ __forceinline__ void load_table(BLds& s, const double2* __restrict__ Us, int node, int box, int tid) {
  for (int e = tid; e < box; e += NTHREADS) s.tb[0][e] = Us[(long long)node * box + e];
}

__global__ __launch_bounds__(NTHREADS, 1) void backward_kernel(BwdArgs a) {
  __shared__ BLds s;
  const int tid = threadIdx.x;
  const int p = blockIdx.x;
  const StructDev S = a.structs[a.pair_struct[p]];
  const int N = S.n_beams;
  const int L = S.n_slices;
  const double h = S.h;
  const int nps = a.nodes_per_slice;
  const double2* __restrict__ Us = a.U + S.table_off;
  const char* pws = a.ws + (long long)p * a.ck.pair_stride;
  double2* __restrict__ ub = a.ubar + (long long)p * a.ubar_stride;
  const int* bptr = a.bin_ptr + S.bin_ptr_off;
  const int* bjk = a.bin_jk + S.bin_jk_off;

  const long long tot = (long long)S.n_nodes * S.box;
  for (long long e = tid; e < tot; e += NTHREADS) ub[e] = make_double2(0.0, 0.0);
  const int W = 2 * S.kd + 1;
  if (tid < NP) {
    const int hh_ = tid < N ? a.beams[2 * (S.beam_off + tid)] : 0;
    const int kk_ = tid < N ? a.beams[2 * (S.beam_off + tid) + 1] : 0;
    s.bhk[tid][0] = hh_;
    s.bhk[tid][1] = kk_;
    s.offk[tid] = hh_ * W + kk_;
    s.basej[tid] = (hh_ + S.hd) * W + kk_ + S.kd;
  }
  if (tid == 0) s.flag_singular = 0;
  if (tid == 0) s.tb[0][S.box] = make_double2(0.0, 0.0);
  __syncthreads();
  const double th0 = a.angles[2 * p], th1 = a.angles[2 * p + 1];
  const double b0x = S.gamma * cos(th0) * cos(th1);
  const double b0y = S.gamma * cos(th0) * sin(th1);
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

  // ---- final step: x = B^{-1} e_1, rho = A x, cotangent of Z_L = y x^H
  const double2* zL = reinterpret_cast<const double2*>(pws + (long long)(a.ck.max_ckpt - 1) * a.ck.state_bytes);
  for (int e = tid; e < NP * NP; e += NTHREADS) {
    const int r = e / NP;
    const double g2v = s.g2s[r];
    const double gr = g2v >= 0.0 ? sqrt(g2v) : 0.0, gi = g2v >= 0.0 ? 0.0 : -sqrt(-g2v);
    const double2 q = zL[e], pp = zL[NP * NP + e];
    const double qr = gr * q.x - gi * q.y, qi = gr * q.y + gi * q.x;
    s.zb[e] = make_double2(qr + pp.y, qi - pp.x);  // B = Gamma Q - iP
    const int c = e - r * NP;
    s.zb[NP * NP + e] = make_double2(r == c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  gauss_jordan(s.zb, s.gj_colp, s.gj_colk, s.gj_rowk, &s.flag_singular, N, tid);
  const double2* Binv = s.zb + NP * NP;
  if (tid < NP) s.x[tid] = tid < N ? Binv[tid * NP + 0] : make_double2(0.0, 0.0);
  __syncthreads();
  // rho = A x with A = Gamma Q + iP (rows < N), into tmp
  {
    const int j = tid >> 2, part = tid & 3;
    double2 acc = make_double2(0.0, 0.0);
    if (j < N) {
      const double g2v = s.g2s[j];
      const double gr = g2v >= 0.0 ? sqrt(g2v) : 0.0, gi = g2v >= 0.0 ? 0.0 : -sqrt(-g2v);
      for (int k = part; k < N; k += 4) {
        const double2 q = zL[j * NP + k], pp = zL[NP * NP + j * NP + k];
        const double2 aj = make_double2(gr * q.x - gi * q.y - pp.y, gr * q.y + gi * q.x + pp.x);
        acc.x += aj.x * s.x[k].x - aj.y * s.x[k].y;
        acc.y += aj.x * s.x[k].y + aj.y * s.x[k].x;
      }
    }
    acc.x += __shfl_xor(acc.x, 1, 64);
    acc.y += __shfl_xor(acc.y, 1, 64);
    acc.x += __shfl_xor(acc.x, 2, 64);
    acc.y += __shfl_xor(acc.y, 2, 64);
    if (part == 0) s.tmp[j] = acc;
  }
  __syncthreads();
  // rho_bar (into tmp2)
  if (tid < NP) {
    double2 rb = make_double2(0.0, 0.0);
    const double gj = s.g2s[tid];
    if (tid < N && gj > 0.0) {
      double wgt = sqrt(s.g2s[0]) / sqrt(gj);
      if (a.convention == 1) wgt *= sin(th0);
      const double sc = 2.0 * wgt * a.dLdI[(long long)p * a.ld + tid];
      rb = make_double2(sc * s.tmp[tid].x, sc * s.tmp[tid].y);
    }
    s.tmp2[tid] = rb;
  }
  __syncthreads();
  // x_bar = A^H rho_bar (into tmp)
  {
    const int k = tid >> 2, part = tid & 3;
    double2 acc = make_double2(0.0, 0.0);
    if (k < N)
      for (int j = part; j < N; j += 4) {
        const double g2v = s.g2s[j];
        const double gr = g2v >= 0.0 ? sqrt(g2v) : 0.0, gi = g2v >= 0.0 ? 0.0 : -sqrt(-g2v);
        const double2 q = zL[j * NP + k], pp = zL[NP * NP + j * NP + k];
        const double2 aj = make_double2(gr * q.x - gi * q.y - pp.y, gr * q.y + gi * q.x + pp.x);
        const double2 t = cmulc(aj, s.tmp2[j]);
        acc.x += t.x;
        acc.y += t.y;
      }
    acc.x += __shfl_xor(acc.x, 1, 64);
    acc.y += __shfl_xor(acc.y, 1, 64);
    acc.x += __shfl_xor(acc.x, 2, 64);
    acc.y += __shfl_xor(acc.y, 2, 64);
    __syncthreads();
    if (part == 0) s.tmp[k] = acc;
  }
  __syncthreads();
  // w = Binv^H x_bar; y = [conj(Gamma)(rho_bar - w); -i (rho_bar + w)]
  {
    const int k = tid >> 2, part = tid & 3;
    double2 acc = make_double2(0.0, 0.0);
    if (k < N)
      for (int j = part; j < N; j += 4) {
        const double2 t = cmulc(Binv[j * NP + k], s.tmp[j]);
        acc.x += t.x;
        acc.y += t.y;
      }
    acc.x += __shfl_xor(acc.x, 1, 64);
    acc.y += __shfl_xor(acc.y, 1, 64);
    acc.x += __shfl_xor(acc.x, 2, 64);
    acc.y += __shfl_xor(acc.y, 2, 64);
    if (part == 0 && k < NP) {
      double2 cbv = make_double2(0.0, 0.0), dbv = make_double2(0.0, 0.0);
      if (k < N) {
        const double g2v = s.g2s[k];
        const double gr = g2v >= 0.0 ? sqrt(g2v) : 0.0, gi = g2v >= 0.0 ? 0.0 : -sqrt(-g2v);
        const double2 rb = s.tmp2[k];
        const double2 dm = make_double2(rb.x - acc.x, rb.y - acc.y);
        cbv = make_double2(gr * dm.x + gi * dm.y, gr * dm.y - gi * dm.x);  // conj(Gamma) (rho_bar - w)
        const double2 sp = make_double2(rb.x + acc.x, rb.y + acc.y);
        dbv = make_double2(sp.y, -sp.x);                                    // -i (rho_bar + w)
      }
      s.cb_[k] = cbv;
      s.db_[k] = dbv;
    }
  }
  __syncthreads();

  // ---- slices, last to first
  for (int i = L - 1; i >= 0; --i) {
    if (pws[a.ck.flags_off + i]) {
      // Through Z' = Z Q^{-1} (with its dependence on Z): the cotangent
      // y' x'^H of Z' = [I; R] becomes y x^H with x = Q^{-1} x' and
      // y = y' - [Z'^H y'; 0] = [-R^H y'_(c'); y'_(c')].  The projection keeps y
      // free of the components that grow under the backward recursion.
      const double2* rz = reinterpret_cast<const double2*>(pws + (long long)(i + 1) * a.ck.state_bytes) + NP * NP;
      matvec_dense_h(rz, s.db_, s.tmp, N, tid);
      __syncthreads();
      if (tid < NP) s.cb_[tid] = make_double2(-s.tmp[tid].x, -s.tmp[tid].y);
      __syncthreads();
      const double2* qs = reinterpret_cast<const double2*>(pws + a.ck.q_off + (long long)i * NP * NP * sizeof(double2));
      invert_into_bottom(s, qs, N, tid);
      matvec_dense(s.zb + NP * NP, s.x, s.tmp, N, tid);  // shared-memory matrix via generic pointer
      __syncthreads();
      if (tid < NP) s.x[tid] = s.tmp[tid];
      __syncthreads();
    }
    // psi = Z_i x
    const double2* zi = reinterpret_cast<const double2*>(pws + (long long)i * a.ck.state_bytes);
    matvec_dense(zi, s.x, s.pc, N, tid);
    matvec_dense(zi + NP * NP, s.x, s.pd, N, tid);
    const int nb = i * nps;
    __syncthreads();
    // RK stages on psi: Y_r = psi + h sum_{j<r} a_rj K_j,  K_r = (Y_r^(c'), -M_r Y_r^(c))
    for (int r = 0; r < a.stages; ++r) {
      if (tid < NP) {
        double2 c = s.pc[tid], dd = s.pd[tid];
        for (int j2 = 0; j2 < r; ++j2) {
          const double ar = a.A[r][j2];
          if (ar != 0.0) {
            c.x += h * ar * s.sv.yd[j2][tid].x;
            c.y += h * ar * s.sv.yd[j2][tid].y;
            dd.x += h * ar * s.sv.kd[j2][tid].x;
            dd.y += h * ar * s.sv.kd[j2][tid].y;
          }
        }
        s.sv.yc[r][tid] = c;
        s.sv.yd[r][tid] = dd;
      }
      load_table(s, Us, nb + a.stage_node[r], S.box, tid);
      __syncthreads();
      matvec_u(s, s.tb[0], s.sv.yc[r], s.tmp, false, N, S.box, tid);
      __syncthreads();
      if (tid < NP) s.sv.kd[r][tid] = make_double2(-s.tmp[tid].x, -s.tmp[tid].y);
      __syncthreads();
    }
    // adjoint of the step, stages last to first
    for (int r = a.stages - 1; r >= 0; --r) {
      if (tid < NP) {
        double2 kc = make_double2(h * a.b[r] * s.cb_[tid].x, h * a.b[r] * s.cb_[tid].y);
        double2 kdb = make_double2(h * a.b[r] * s.db_[tid].x, h * a.b[r] * s.db_[tid].y);
        for (int m = r + 1; m < a.stages; ++m) {
          const double am = a.A[m][r];
          if (am != 0.0) {
            kc.x += h * am * s.sv.ybc[m][tid].x;
            kc.y += h * am * s.sv.ybc[m][tid].y;
            kdb.x += h * am * s.sv.ybd[m][tid].x;
            kdb.y += h * am * s.sv.ybd[m][tid].y;
          }
        }
        s.sv.ybd[r][tid] = kc;   // Y_bar^(c') of stage r = K_bar^(c)
        s.tmp2[tid] = kdb;    // K_bar^(c') of stage r
      }
      load_table(s, Us, nb + a.stage_node[r], S.box, tid);
      __syncthreads();
      matvec_u(s, s.tb[0], s.tmp2, s.tmp, true, N, S.box, tid);
      __syncthreads();
      if (tid < NP) s.sv.ybc[r][tid] = make_double2(-s.tmp[tid].x, -s.tmp[tid].y);
      // dL/dU at this stage's node: sum over (j,k) of a rod difference of
      // g_j conj(v_k) with g = -K_bar^(c'), v = Y_r^(c)
      double2* un = ub + (long long)(nb + a.stage_node[r]) * S.box;
      for (int bin = tid; bin < S.box; bin += NTHREADS) {
        double2 acc = make_double2(0.0, 0.0);
        for (int t = bptr[bin]; t < bptr[bin + 1]; ++t) {
          const int jk = bjk[t];
          const int j = jk / NP, k = jk - j * NP;
          const double2 g = s.tmp2[j];
          const double2 v = s.sv.yc[r][k];
          // -g * conj(v)
          acc.x -= g.x * v.x + g.y * v.y;
          acc.y -= g.y * v.x - g.x * v.y;
        }
        const double2 o = un[bin];
        un[bin] = make_double2(o.x + acc.x, o.y + acc.y);
      }
      __syncthreads();
    }
    if (tid < NP) {
      double2 c = s.cb_[tid], dd = s.db_[tid];
      for (int r = 0; r < a.stages; ++r) {
        c.x += s.sv.ybc[r][tid].x;
        c.y += s.sv.ybc[r][tid].y;
        dd.x += s.sv.ybd[r][tid].x;
        dd.y += s.sv.ybd[r][tid].y;
      }
      s.cb_[tid] = c;
      s.db_[tid] = dd;
    }
    __syncthreads();
  }
}

// dL/dU of structure s = sum over its pairs of the per-pair tables (fixed order).
__global__ __launch_bounds__(256) void reduce_ubar_kernel(ReduceArgs a) {
  const StructDev S = a.structs[blockIdx.y];
  const long long tot = (long long)S.n_nodes * S.box;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= tot) return;
  double2 acc = make_double2(0.0, 0.0);
  for (int q = 0; q < S.n_angles; ++q) {
    const double2 v = a.ubar[(long long)(S.pair_off + q) * a.ubar_stride + e];
    acc.x += v.x;
    acc.y += v.y;
  }
  a.dU[S.table_off + e] = acc;
}

hipError_t launch_backward(const BwdArgs& a, hipStream_t stream) {
  hipLaunchKernelGGL(backward_kernel, dim3(a.n_pairs), dim3(NTHREADS), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_reduce_ubar(const ReduceArgs& a, int n_struct, long long max_table, hipStream_t stream) {
  hipLaunchKernelGGL(reduce_ubar_kernel, dim3((unsigned)((max_table + 255) / 256), n_struct), dim3(256), 0, stream, a);
  return hipGetLastError();
}

}  // namespace rheed
