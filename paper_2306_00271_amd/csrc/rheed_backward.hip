// Adjoint of the forward propagation (not in the paper), on gfx950.
//
// Only the first column of the reflection matrix is used (rho(0) = R e_1,
// Algorithm 1), so the cotangent of every intermediate state is rank one:
// if the final state Z_L has cotangent y x^H, then
//   * through a slice map Z <- Phi Z (an RK step is linear from the left)
//     the cotangent becomes (Phi^H y) x^H;
//   * through a right-hand-side transformation Z' = Z Q^{-1} (Sec. 3.2) it
//     becomes y x^H with x = Q^{-1} x' and y = y' - [Z'^H y'; 0] =
//     [-R^H y'_(c'); y'_(c')] for Z' = [I; R]; the second term is the
//     derivative of Q^{-1} itself.  The output is invariant under right
//     multiplication of Z, so in exact arithmetic that term changes nothing,
//     but it removes the components of y that the backward recursion would
//     amplify;
//   * the gradient of the coupling matrix at stage r is g_r v_r^H with v_r the
//     stage input of the RK step applied to the single physical column
//     psi = Z x, and g_r = -K_bar_r^(c') the adjoint of that stage's product.
// One workgroup per (structure, angle) pair therefore walks the slices
// backwards with vectors only.  The forward pass keeps Z at the start of every
// K-th slice, T = Q^{-1} of every transformation and, for K > 1, R (the
// normalised P after it).  Per K-slice segment, from the top: x is carried
// down through the segment's transformations, psi = Z x is formed at the
// segment's stored state and stepped up through the segment by the RK step
// (psi = Z x is unchanged by Z <- Z T, x <- T^{-1} x), and the adjoint then
// walks back down.  Each stage costs one N x N matrix-vector product against
// the node's rod-difference table in LDS.  Every stage writes (v_r, g_r) to a stage buffer;
// grad_assemble_kernel then sums g v^H over the angles and stages of each
// node on the FP64 matrix cores and bins the sum by rod difference, in a
// fixed order.
//
// Thread layout of the vector work, for states padded to W = 64 (N <= 64) or
// W = 128 (64 < N <= 128): W / 8 waves, thread t works on row j = t >> 3 and
// on columns (W / 8) (t & 7) .. +W/8-1; the eight threads of a row reduce by
// butterflies and all hold the row's result.  With W = 64 the final step
// inverts B itself (register Gauss-Jordan); with W = 128 the forward pass
// keeps B^{-1} beside the final state.
//
// Final step (Eq. vrhocomp, first column): with B = Gamma Q - iP,
// A = Gamma Q + iP, B x = e_1, rho = A x and
// eta_j = w_j |rho_j|^2 (w_j = Gamma_0/Gamma_j on open beams, times sin theta0
// in the printed normalisation):
//   rho_bar_j = 2 w_j rho_j dL/deta_j,  x_bar = A^H rho_bar,  w = B^{-H} x_bar,
//   cotangent of Z_L = [conj(Gamma)(rho_bar - w); -i (rho_bar + w)] x^H.
#include "rheed_internal.h"
#include "rheed_gj.h"
#include "rheed_large.h"

namespace rheed {

// Launch geometry of the adjoint for the state width W of its pairs (64 for
// N <= 64, 128 for 64 < N <= 128, 256 above): tpr threads per row (8, or 4
// at W = 256), thread t works on row j = t / tpr and on W / tpr of its
// columns (the threads of a row reduce by butterflies and all hold the
// row's result).  At W = 256 the gather indices of the table come from
// per-beam offsets in LDS instead of registers.
template <int W>
struct BGeo {
  static constexpr int tpr = W == NX ? 4 : 8;
  static constexpr int threads = W * tpr;
  static constexpr int waves = threads / 64;
  static constexpr int cols = W / tpr;
  static constexpr bool idx_regs = W != NX;
  static constexpr int box = W == NP ? MAXBOX : W == NL ? MAXBOXL : MAXBOXX;  // table row entries in LDS
  // node-table slots: with W = 64 the current slice's (nps + 1) and the next
  // one's (nps) for the RK steppers, or a splitting method's nps + 1 <= 13
  // kick positions; with W = 128 only the current slice's (LDS), so the next
  // slice's tables go in after the current one's last product
  static constexpr int ring = W == NP ? 13 : 5;
  static constexpr int pf = (4 * box + threads - 1) / threads;  // prefetch registers for nps <= 4 nodes
};

// Explicit RK tableaux (Sec. 3.4).  node[r] is the table node of stage r
// counted from the slice's c = 0 node (nps = the next slice's c = 0).
template <int S>
struct BTab;
template <>
struct BTab<0> {  // classical RK4, c = 0, 1/2, 1/2, 1
  static constexpr int stages = 4, nps = 2;
  static constexpr int node[4] = {0, 1, 1, 2};
  static constexpr double a[4][4] = {{0, 0, 0, 0}, {0.5, 0, 0, 0}, {0, 0.5, 0, 0}, {0, 0, 1, 0}};
  static constexpr double b[4] = {1.0 / 6, 1.0 / 3, 1.0 / 3, 1.0 / 6};
};
template <>
struct BTab<2> {  // a splitting method: its kicks and drifts come with the launch (BwdArgs::sp)
  static constexpr int stages = 1, nps = 1;
  static constexpr int node[1] = {0};
  static constexpr double a[1][1] = {{0}};
  static constexpr double b[1] = {0};
};
template <>
struct BTab<1> {  // Butcher's 6th order, 7 stages, c = 0, 1/3, 2/3, 1/3, 1/2, 1/2, 1
  static constexpr int stages = 7, nps = 4;
  static constexpr int node[7] = {0, 1, 3, 1, 2, 2, 4};
  static constexpr double a[7][7] = {
      {0, 0, 0, 0, 0, 0, 0},
      {1.0 / 3, 0, 0, 0, 0, 0, 0},
      {0, 2.0 / 3, 0, 0, 0, 0, 0},
      {1.0 / 12, 1.0 / 3, -1.0 / 12, 0, 0, 0, 0},
      {-1.0 / 16, 9.0 / 8, -3.0 / 16, -3.0 / 8, 0, 0, 0},
      {0, 9.0 / 8, -3.0 / 8, -3.0 / 4, 1.0 / 2, 0, 0},
      {9.0 / 44, -9.0 / 11, 63.0 / 44, 18.0 / 11, 0, -16.0 / 11, 0}};
  static constexpr double b[7] = {11.0 / 120, 0, 27.0 / 40, 27.0 / 40, -4.0 / 15, -4.0 / 15, 11.0 / 120};
};

template <int W>
struct BLds {
  double2 tb[BGeo<W>::ring][BGeo<W>::box + 1];  // node tables; entry `box` of every slot stays 0
  double2 vin[2][W];             // matrix-vector inputs (double buffered: one barrier per product)
  double2 x[W];                  // coefficients of the physical column
  double2 red[W == NP ? BGeo<W>::waves : 1][W];  // W = 64: per-wave partial sums
  double2 gj_row[2 * NP];        // W = 64: the elimination of the final step
  int gj_piv[NP];
  double g2s[W];
  int bhk[W][2];
  int sbase[W == NX ? W : 1];    // W = 256: (h_j + hd)(2 kd + 1) + k_j + kd and h_j (2 kd + 1) + k_j of beam j
  int soff[W == NX ? W : 1];
  int flag_singular;
};


__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 caxpy(double s, double2 x, double2 y) {  // y + s x
  return make_double2(y.x + s * x.x, y.y + s * x.y);
}

// v from another lane of the same row of 8, by DPP (CTRL: a quad_perm or
// row_half_mirror pattern).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xf, 0xf, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the TPR threads of a row (8: lanes 8r .. 8r+7, 4: lanes 4r ..
// 4r+3): pairs, then quads (quad_perm), then for eight the two quads
// (row_half_mirror); every lane of the row ends with the same sum.
template <int TPR = 8>
__device__ __forceinline__ double2 row_sum(double2 v) {
  v.x += dpp_f64<0xB1>(v.x);
  v.y += dpp_f64<0xB1>(v.y);
  v.x += dpp_f64<0x4E>(v.x);
  v.y += dpp_f64<0x4E>(v.y);
  if constexpr (TPR == 8) {
    v.x += dpp_f64<0x141>(v.x);
    v.y += dpp_f64<0x141>(v.y);
  }
  return v;
}

// (M v)_j (HERM = false) or (M^H v)_j (HERM = true), M = U(node) + Gamma^2;
// ix[q] is the table entry of U_{j,k} (or U_{k,j}) for
// k = C part + ((q + part) mod C), C = W / 8 columns per thread, or `box`
// (a zero entry) outside the n x n block.
// With W = 256 (IX = false) the entry is formed per column from the offsets
// in LDS: U_{j,k} at sbase_j - soff_k, U_{k,j} at sbase_k - soff_j.
template <bool HERM, int W, bool IX = BGeo<W>::idx_regs>
__device__ __forceinline__ double2 matvec_row(const double2* __restrict__ tslot, const double2* __restrict__ v,
                                              const int (&ix)[IX ? BGeo<W>::cols : 1], int part, int j, double g2j,
                                              const int* sbase = nullptr, const int* soff = nullptr, int n = 0,
                                              int box = 0) {
  constexpr int C = BGeo<W>::cols;
  double2 a0 = make_double2(0.0, 0.0), a1 = make_double2(0.0, 0.0);
#pragma unroll 4
  for (int h = 0; h < C; h += 4) {  // four products' operands in flight at a time
    double2 u[4], vk[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = C * part + ((h + q + part) & (C - 1));
      if constexpr (IX) {
        u[q] = tslot[ix[h + q]];
      } else {
        const bool in = j < n && k < n;
        u[q] = tslot[in ? (HERM ? sbase[k] - soff[j] : sbase[j] - soff[k]) : box];
      }
      vk[q] = v[k];
    }
#pragma unroll
    for (int q = 0; q < 4; q += 2) {
      a0 = cadd(a0, HERM ? cmulc(u[q], vk[q]) : cmul(u[q], vk[q]));
      a1 = cadd(a1, HERM ? cmulc(u[q + 1], vk[q + 1]) : cmul(u[q + 1], vk[q + 1]));
    }
  }
  const double2 vj = v[j];
  const double2 acc = row_sum<BGeo<W>::tpr>(cadd(a0, a1));
  return make_double2(acc.x + g2j * vj.x, acc.y + g2j * vj.y);
}

// The adjoint of one pair's forward pass in two workgroups (roles), W the
// padded width of its stored states (64 or 128).
template <int STEPPER, int W>
__global__ __launch_bounds__(BGeo<W>::threads, 1) void backward_kernel(BwdArgs a) {
  using T = BTab<STEPPER>;
  using G = BGeo<W>;
  constexpr int NS = T::stages;
  constexpr int NPS = T::nps;
  constexpr int BW = G::waves, BT = G::threads, CP = G::cols, RING = G::ring, PF = G::pf, TPR = G::tpr;
  constexpr bool IXR = G::idx_regs;
  // the next slice's tables overwrite slots the current slice still reads
  constexpr bool tight = RING < 2 * NPS + 1;
  __shared__ BLds<W> s;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int j = tid / TPR, part = tid % TPR;
  // two workgroups per pair: role 0 carries x down and psi up and writes the
  // stage inputs v_r, role 1 walks the adjoint stages down and writes g_r;
  // the two need nothing from each other
  const int role = blockIdx.x & 1;
  const int p = a.pair_list ? a.pair_list[blockIdx.x >> 1] : (int)(blockIdx.x >> 1);
  const StructDev S = a.structs[a.pair_struct[p]];
  const int N = S.n_beams;
  const int L = S.n_slices;
  const int box = S.box;
  const double h = S.h;
  const double2* __restrict__ Us = a.U + S.table_off;
  const char* pws = a.ws + (long long)p * a.ck.pair_stride;
  const char* flags = pws + a.ck.flags_off;
  double2* __restrict__ gb = a.gbuf + (long long)p * a.g_pair_stride;
  constexpr long long MATB = (long long)W * W * sizeof(double2);

  if (tid < W) {
    s.bhk[tid][0] = tid < N ? a.beams[2 * (S.beam_off + tid)] : 0;
    s.bhk[tid][1] = tid < N ? a.beams[2 * (S.beam_off + tid) + 1] : 0;
  }
  if (tid < RING) s.tb[tid][box] = make_double2(0.0, 0.0);
  if (tid == 0) s.flag_singular = 0;
  __syncthreads();
  const double th0 = a.angles[2 * p], th1 = a.angles[2 * p + 1];
  if (tid < W) {
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
  // table entries of U_{j,k} (role 0) or U_{k,j} (role 1) for
  // k = CP part + ((q + part) mod CP): the eight threads of a row visit their
  // columns in rotated order, so that their reads of the input vector fall in
  // different LDS bank groups
  int ix[IXR ? CP : 1];
  if constexpr (IXR) {
    const int Wd = 2 * S.kd + 1;
#pragma unroll 8
    for (int q = 0; q < CP; ++q) {
      const int k = CP * part + ((q + part) & (CP - 1));
      const bool in = j < N && k < N;
      const int bj = (s.bhk[j][0] + S.hd) * Wd + s.bhk[j][1] + S.kd, oj = s.bhk[j][0] * Wd + s.bhk[j][1];
      const int bk = (s.bhk[k][0] + S.hd) * Wd + s.bhk[k][1] + S.kd, ok = s.bhk[k][0] * Wd + s.bhk[k][1];
      ix[q] = in ? (role == 0 ? bj - ok : bk - oj) : box;
    }
  } else {
    ix[0] = 0;
    if (tid < W) {
      const int Wd = 2 * S.kd + 1;
      s.sbase[tid] = (s.bhk[tid][0] + S.hd) * Wd + s.bhk[tid][1] + S.kd;
      s.soff[tid] = s.bhk[tid][0] * Wd + s.bhk[tid][1];
    }
  }
  __syncthreads();
  const double g2j = s.g2s[j];
  // the product of a stage: (M v)_j (role 0) or (M^H v)_j (role 1) with the table in tslot
  auto mv_f = [&](const double2* tslot, const double2* v) {
    if constexpr (IXR) return matvec_row<false, W>(tslot, v, ix, part, j, g2j);
    else return matvec_row<false, W>(tslot, v, ix, part, j, g2j, s.sbase, s.soff, N, box);
  };
  auto mv_h = [&](const double2* tslot, const double2* v) {
    if constexpr (IXR) return matvec_row<true, W>(tslot, v, ix, part, j, g2j);
    else return matvec_row<true, W>(tslot, v, ix, part, j, g2j, s.sbase, s.soff, N, box);
  };

  // ---- final step: x = B^{-1} e_1, rho = A x
  const double2* zL = reinterpret_cast<const double2*>(pws + (long long)(a.ck.max_ckpt - 1) * a.ck.state_bytes);
  double2 yc, yd;  // cotangent of row j of the current state
  {
    // W = 64: B^{-1} by elimination here; slot sl = w + BW (m - 8) < N of
    // z holds row gj_piv[sl] of B^{-1}, column pos in this lane.  W = 128:
    // B^{-1} as the forward pass kept it.
    double2 z[16];
    int pos = 0;
    const double2* Binv = reinterpret_cast<const double2*>(pws + a.ck.binv_off);
    if constexpr (W == NP) {
      if (tid < W) s.x[tid] = make_double2(0.0, 0.0);
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int r = w + BW * m;
        const double g2v = s.g2s[r];
        const double gr = g2v >= 0.0 ? sqrt(g2v) : 0.0, gi = g2v >= 0.0 ? 0.0 : -sqrt(-g2v);
        const double2 q = zL[r * W + lane], pp = zL[W * W + r * W + lane];
        z[m] = make_double2(gr * q.x - gi * q.y + pp.y, gr * q.y + gi * q.x - pp.x);  // Gamma Q - iP
      }
      pos = gj_inverse<BW>(z, N, lane, w, s.gj_row, s.gj_piv, &s.flag_singular);
      if (pos == 0) {
#pragma unroll
        for (int m = 8; m < 16; ++m) {
          const int sl = w + BW * (m - 8);
          if (sl < N) s.x[s.gj_piv[sl]] = z[m];
        }
      }
    } else {
      if (part == 0) s.x[j] = j < N ? Binv[(long long)j * W] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    // rho_j = sum_k A[j][k] x_k, A = Gamma Q + iP
    double2 rho;
    {
      const double gr = g2j >= 0.0 ? sqrt(g2j) : 0.0, gi = g2j >= 0.0 ? 0.0 : -sqrt(-g2j);
      double2 acc = make_double2(0.0, 0.0);
#pragma unroll 8
      for (int q = 0; q < CP; ++q) {
        const int k = CP * part + q;
        const double2 qv = zL[j * W + k], pv = zL[W * W + j * W + k];
        const double2 av = make_double2(gr * qv.x - gi * qv.y - pv.y, gr * qv.y + gi * qv.x + pv.x);
        acc = cadd(acc, cmul(av, s.x[k]));
      }
      rho = row_sum<TPR>(acc);
    }
    // rho_bar
    double2 rb = make_double2(0.0, 0.0);
    if (j < N && g2j > 0.0) {
      double wgt = sqrt(s.g2s[0]) / sqrt(g2j);
      if (a.convention == 1) wgt *= sin(th0);
      const double sc = 2.0 * wgt * a.dLdI[(long long)p * a.ld + j];
      rb = make_double2(sc * rho.x, sc * rho.y);
    }
    if (part == 0) s.vin[0][j] = rb;
    __syncthreads();
    // x_bar_k = sum_j conj(A[j][k]) rho_bar_j
    double2 xbar;
    {
      const int k = j;
      double2 acc = make_double2(0.0, 0.0);
#pragma unroll 8
      for (int q = 0; q < CP; ++q) {
        const int jj = CP * part + q;
        const double g2v = s.g2s[jj];
        const double gr = g2v >= 0.0 ? sqrt(g2v) : 0.0, gi = g2v >= 0.0 ? 0.0 : -sqrt(-g2v);
        const double2 qv = zL[jj * W + k], pv = zL[W * W + jj * W + k];
        const double2 av = make_double2(gr * qv.x - gi * qv.y - pv.y, gr * qv.y + gi * qv.x + pv.x);
        acc = cadd(acc, cmulc(av, s.vin[0][jj]));
      }
      xbar = row_sum<TPR>(acc);
    }
    if (part == 0) s.vin[1][j] = xbar;
    __syncthreads();
    // w_k = sum_j conj(Binv[j][k]) xbar_j
    double2 wv = make_double2(0.0, 0.0);
    if constexpr (W == NP) {
      // this lane holds column pos of the rows in its slots
      double2 acc = make_double2(0.0, 0.0);
#pragma unroll
      for (int m = 8; m < 16; ++m) {
        const int sl = w + BW * (m - 8);
        if (sl < N) acc = cadd(acc, cmulc(z[m], s.vin[1][s.gj_piv[sl]]));
      }
      s.red[w][pos] = acc;
      __syncthreads();
#pragma unroll
      for (int q = 0; q < BW; ++q) wv = cadd(wv, s.red[q][j]);
    } else {
      double2 acc = make_double2(0.0, 0.0);
#pragma unroll 8
      for (int q = 0; q < CP; ++q) {
        const int jj = CP * part + q;
        acc = cadd(acc, cmulc(Binv[(long long)jj * W + j], s.vin[1][jj]));
      }
      wv = row_sum<TPR>(acc);
    }
    yc = make_double2(0.0, 0.0);
    yd = make_double2(0.0, 0.0);
    if (j < N) {
      const double gr = g2j >= 0.0 ? sqrt(g2j) : 0.0, gi = g2j >= 0.0 ? 0.0 : -sqrt(-g2j);
      const double2 dm = make_double2(rb.x - wv.x, rb.y - wv.y);
      yc = make_double2(gr * dm.x + gi * dm.y, gr * dm.y - gi * dm.x);  // conj(Gamma) (rho_bar - w)
      const double2 sp = make_double2(rb.x + wv.x, rb.y + wv.y);
      yd = make_double2(sp.y, -sp.x);                                    // -i (rho_bar + w)
    }
    __syncthreads();
  }

  const int K = a.ck.every;
  auto load_tables = [&](int i) {  // nodes of slice i, in their ring slots
    for (int e = tid; e < (NPS + 1) * box; e += BT) {
      const int nn = i * NPS + e / box;
      s.tb[nn % RING][e % box] = Us[(long long)nn * box + e % box];
    }
  };
  // splitting methods: the nodes of slice i (positions 0 .. nps) in ring slots 0 .. nps
  auto load_slice_nodes = [&](int i, int count) {
    const int nps = a.sp.nps;
    for (int e = tid; e < count * box; e += BT) {
      const int q = e / box;
      s.tb[q][e - q * box] = Us[(long long)(i * nps + q) * box + e - q * box];
    }
  };
  const int NKS = STEPPER == 2 ? (a.sp.form == 0 ? a.sp.kicks - 1 : a.sp.kicks) : NS;  // kicks kept per slice
  if (role == 0) {
    if constexpr (STEPPER == 2) {
      if (a.sp.form == 0) {
        // v of the BAB method's final kick (after the last slice): the c part of
        // psi = Z_L x at the final state, which that kick does not change
        double2 ac = make_double2(0.0, 0.0);
#pragma unroll 8
        for (int q = 0; q < CP; ++q) ac = cadd(ac, cmul(zL[j * W + CP * part + q], s.x[CP * part + q]));
        ac = row_sum<TPR>(ac);
        if (part == 0) gb[(long long)L * NKS * 2 * W + j] = ac;
      }
    }
    // Segments of K = ck.every slices, from the top down.  (A) x moves down
    // through the segment's transformations, x <- T_m x for every slice m
    // whose decision byte is set; (B) psi_lo = Z_lo x_lo from the stored
    // state, then psi goes up slice by slice with the RK step itself
    // (psi_{i+1} = Phi_i psi_i: psi = Z x does not change under Z <- Z T,
    // x <- T^{-1} x), the stage inputs v_r going to the stage buffer.
    for (int hi = L; hi > 0;) {
      const int lo = ((hi - 1) / K) * K;
      // (A) x down to the bottom of the segment; x at each transformed state
      // inside the segment is kept for (B)
      double2* xs = a.xs + (long long)p * a.xs_stride;
      for (int m = hi - 1; m >= lo; --m) {
        if (flags[m]) {
          if (K > 1 && m + 1 < hi && tid < W) xs[(m + 1 - lo) * W + tid] = s.x[tid];
          const double2* Tm = reinterpret_cast<const double2*>(pws + a.ck.q_off + (long long)m * MATB);
          double2 xn = make_double2(0.0, 0.0);
#pragma unroll 8
          for (int q = 0; q < CP; ++q) xn = cadd(xn, cmul(Tm[j * W + CP * part + q], s.x[CP * part + q]));
          xn = row_sum<TPR>(xn);
          __syncthreads();
          if (part == 0) s.x[j] = xn;
          __syncthreads();
        }
      }
      // (B) psi_lo = Z_lo x_lo, then up through the segment; at a state that a
      // transformation left as [I; R], psi = [I; R] x is formed afresh, so the
      // RK step carries psi only across well-conditioned stretches
      double2 psic, psid;
      {
        const double2* z = reinterpret_cast<const double2*>(pws + (long long)(lo / K) * a.ck.state_bytes);
        double2 ac = make_double2(0.0, 0.0), ad = make_double2(0.0, 0.0);
#pragma unroll 8
        for (int q = 0; q < CP; ++q) {
          const double2 xk = s.x[CP * part + q];
          ac = cadd(ac, cmul(z[j * W + CP * part + q], xk));
          ad = cadd(ad, cmul(z[W * W + j * W + CP * part + q], xk));
        }
        psic = row_sum<TPR>(ac);
        psid = row_sum<TPR>(ad);
      }
      if constexpr (STEPPER == 2) {
        // psi through the segment's kicks and drifts; v_k = psi_c at kick k
        const SplitSteps& sp = a.sp;
        for (int i = lo; i < hi; ++i) {
          if (i > lo && flags[i - 1]) {
            const double2* R = reinterpret_cast<const double2*>(pws + a.ck.r_off + (long long)(i - 1) * MATB);
            const double2* xi = xs + (i - lo) * W;
            double2 ad = make_double2(0.0, 0.0);
#pragma unroll 8
            for (int q = 0; q < CP; ++q) ad = cadd(ad, cmul(R[j * W + CP * part + q], xi[CP * part + q]));
            psic = xi[j];
            psid = row_sum<TPR>(ad);
          }
          __syncthreads();  // the previous slice's products are done with the ring
          load_slice_nodes(i, sp.nps + 1);
          __syncthreads();
          double2* gs = gb + (long long)i * NKS * 2 * W;
          // kick k: v_k = psi_c, psi_d -= h w M(node) psi_c
          auto kick_up = [&](int k, int node, double wgt) {
            if (part == 0) {
              s.vin[k & 1][j] = psic;
              gs[k * 2 * W + j] = psic;
            }
            __syncthreads();
            const double2 mv = mv_f(s.tb[node], s.vin[k & 1]);
            psid = caxpy(-h * wgt, mv, psid);
          };
          if (sp.form == 0) {
            kick_up(0, sp.node[0], i == 0 ? sp.b[0] : sp.b[0] + sp.b[sp.kicks - 1]);
            for (int r = 0; r + 1 < sp.kicks; ++r) {
              psic = caxpy(h * sp.a[r], psid, psic);
              if (r + 2 < sp.kicks) kick_up(r + 1, sp.node[r + 1], sp.b[r + 1]);
            }
          } else {
            psic = caxpy(h * sp.a[0], psid, psic);
            for (int r = 0; r < sp.kicks; ++r) {
              kick_up(r, sp.node[r], sp.b[r]);
              psic = caxpy(h * sp.a[r + 1], psid, psic);
            }
          }
        }
        hi = lo;
        continue;
      }
      __syncthreads();  // the previous segment's last products are done with the ring
      load_tables(lo);
      __syncthreads();
      for (int i = lo; i < hi; ++i) {
        const int nb = i * NPS;
        if (i > lo && flags[i - 1]) {
          const double2* R = reinterpret_cast<const double2*>(pws + a.ck.r_off + (long long)(i - 1) * MATB);
          const double2* xi = xs + (i - lo) * W;
          double2 ad = make_double2(0.0, 0.0);
#pragma unroll 8
          for (int q = 0; q < CP; ++q) ad = cadd(ad, cmul(R[j * W + CP * part + q], xi[CP * part + q]));
          psic = xi[j];
          psid = row_sum<TPR>(ad);
        }
        double2 pf[PF];  // the next slice's new nodes, loaded during this one
        if (i + 1 < hi) {
#pragma unroll
          for (int t = 0; t < PF; ++t) {
            const int e = tid + BT * t;
            if (e < NPS * box) pf[t] = Us[(long long)(nb + NPS + 1) * box + e];
          }
        }
        // RK stages on psi: Y_r = psi + h sum_{m<r} a_rm K_m, K_r = (Y_r^(c'), -M_r Y_r^(c))
        double2* gs = gb + (long long)i * NS * 2 * W;
        double2 Yd[NS], Kd[NS];
#pragma unroll
        for (int r = 0; r < NS; ++r) {
          double2 yr = psic, ydr = psid;
#pragma unroll
          for (int m = 0; m < r; ++m) {
            if (T::a[r][m] != 0.0) {
              yr = caxpy(h * T::a[r][m], Yd[m], yr);
              ydr = caxpy(h * T::a[r][m], Kd[m], ydr);
            }
          }
          Yd[r] = ydr;
          if (part == 0) {
            s.vin[r & 1][j] = yr;
            gs[r * 2 * W + j] = yr;  // v_r
          }
          __syncthreads();
          const double2 mv = mv_f(s.tb[(nb + T::node[r]) % RING], s.vin[r & 1]);
          Kd[r] = make_double2(-mv.x, -mv.y);
        }
        if (i + 1 < hi) {
#pragma unroll
          for (int r = 0; r < NS; ++r) {
            if (T::b[r] != 0.0) {
              psic = caxpy(h * T::b[r], Yd[r], psic);
              psid = caxpy(h * T::b[r], Kd[r], psid);
            }
          }
          if constexpr (tight) __syncthreads();
#pragma unroll
          for (int t = 0; t < PF; ++t) {
            const int e = tid + BT * t;
            if (e < NPS * box) {
              const int q = e / box;
              s.tb[(nb + NPS + 1 + q) % RING][e - q * box] = pf[t];
            }
          }
        }
      }
      hi = lo;
    }
  } else if constexpr (STEPPER == 2) {
    // Down through every slice of a splitting method: the adjoint of a kick
    // c' -= h w M c is y_c -= h w M^H y_d (its g = -h w y_d to the stage
    // buffer), of a drift c += h a c' it is y_d += h a y_c; the projection
    // y_c = -R^H y_d wherever a transformation followed the slice (R from its
    // slot: a splitting method always keeps it).
    const SplitSteps& sp = a.sp;
    auto kick_down = [&](int k, double2* gs, int node, double wgt) {
      const int buf = k & 1;
      if (part == 0) {
        s.vin[buf][j] = yd;
        gs[k * 2 * W + W + j] = make_double2(-h * wgt * yd.x, -h * wgt * yd.y);
      }
      __syncthreads();
      const double2 mv = mv_h(s.tb[node], s.vin[buf]);
      yc = caxpy(-h * wgt, mv, yc);
    };
    if (sp.form == 0) {  // the final kick, at node L nps
      load_slice_nodes(L, 1);
      __syncthreads();
      kick_down(0, gb + (long long)L * NKS * 2 * W, 0, sp.b[sp.kicks - 1]);
    }
    for (int i = L - 1; i >= 0; --i) {
      if (flags[i]) {
        const double2* R = reinterpret_cast<const double2*>(pws + a.ck.r_off + (long long)i * MATB);
        __syncthreads();
        if (part == 0) s.vin[0][j] = yd;
        __syncthreads();
        double2 t = make_double2(0.0, 0.0);
#pragma unroll 8
        for (int q = 0; q < CP; ++q) t = cadd(t, cmulc(R[(CP * part + q) * W + j], s.vin[0][CP * part + q]));
        t = row_sum<TPR>(t);
        yc = make_double2(-t.x, -t.y);
      }
      __syncthreads();  // the previous slice's products are done with the ring and vin
      load_slice_nodes(i, sp.nps + 1);
      __syncthreads();
      double2* gs = gb + (long long)i * NKS * 2 * W;
      if (sp.form == 0) {
        for (int r = sp.kicks - 2; r >= 0; --r) {
          yd = caxpy(h * sp.a[r], yc, yd);
          kick_down(r, gs, sp.node[r], r == 0 ? (i == 0 ? sp.b[0] : sp.b[0] + sp.b[sp.kicks - 1]) : sp.b[r]);
        }
      } else {
        yd = caxpy(h * sp.a[sp.kicks], yc, yd);
        for (int r = sp.kicks - 1; r >= 0; --r) {
          kick_down(r, gs, sp.node[r], sp.b[r]);
          yd = caxpy(h * sp.a[r], yc, yd);
        }
      }
    }
  } else {
    // Down through every slice: the projection y_c = -R^H y_d wherever a
    // transformation followed the slice (R the normalised P after it: the
    // stored state for K = 1, the R slot otherwise), then the adjoint of the
    // slice's RK step, stages last to first, its g_r going to the stage buffer.
    load_tables(L - 1);
    __syncthreads();
    for (int i = L - 1; i >= 0; --i) {
      const int nb = i * NPS;
      double2 pf[PF];  // the new nodes of slice i - 1
      if (i > 0) {
#pragma unroll
        for (int t = 0; t < PF; ++t) {
          const int e = tid + BT * t;
          if (e < NPS * box) pf[t] = Us[(long long)(nb - NPS) * box + e];
        }
      }
      if (flags[i]) {
        const double2* R =
            K == 1 ? (i + 1 == L ? zL : reinterpret_cast<const double2*>(pws + (long long)(i + 1) * a.ck.state_bytes)) +
                         W * W
                   : reinterpret_cast<const double2*>(pws + a.ck.r_off + (long long)i * MATB);
        if (part == 0) s.vin[0][j] = yd;
        __syncthreads();
        double2 t = make_double2(0.0, 0.0);
#pragma unroll 8
        for (int q = 0; q < CP; ++q) t = cadd(t, cmulc(R[(CP * part + q) * W + j], s.vin[0][CP * part + q]));
        t = row_sum<TPR>(t);
        yc = make_double2(-t.x, -t.y);
        __syncthreads();
      }
      double2* gs = gb + (long long)i * NS * 2 * W;
      double2 Ybc[NS], Ybd[NS];
#pragma unroll
      for (int r = NS - 1; r >= 0; --r) {
        double2 kc = make_double2(h * T::b[r] * yc.x, h * T::b[r] * yc.y);
        double2 kd = make_double2(h * T::b[r] * yd.x, h * T::b[r] * yd.y);
#pragma unroll
        for (int m = r + 1; m < NS; ++m) {
          if (T::a[m][r] != 0.0) {
            kc = caxpy(h * T::a[m][r], Ybc[m], kc);
            kd = caxpy(h * T::a[m][r], Ybd[m], kd);
          }
        }
        Ybd[r] = kc;  // Y_bar^(c') = K_bar^(c)
        const int buf = (r + 1) & 1;  // the products alternate between the two input buffers
        if (part == 0) {
          s.vin[buf][j] = kd;
          gs[r * 2 * W + W + j] = make_double2(-kd.x, -kd.y);  // g_r = -K_bar^(c')
        }
        __syncthreads();
        const double2 mv = mv_h(s.tb[(nb + T::node[r]) % RING], s.vin[buf]);
        Ybc[r] = make_double2(-mv.x, -mv.y);  // Y_bar^(c) = -M^H K_bar^(c')
      }
#pragma unroll
      for (int r = 0; r < NS; ++r) {
        yc = cadd(yc, Ybc[r]);
        yd = cadd(yd, Ybd[r]);
      }
      if (i > 0) {
        if constexpr (tight) __syncthreads();
#pragma unroll
        for (int t = 0; t < PF; ++t) {
          const int e = tid + BT * t;
          if (e < NPS * box) {
            const int q = e / box;
            s.tb[(nb - NPS + q) % RING][e - q * box] = pf[t];
          }
        }
      }
      __syncthreads();
    }
  }
}

// dL/dU of node n of structure s: sum over the angles of s and over the
// stages that use node n of g v^H, binned by rod difference:
//   dU[n][d] = sum_{(j,k): g_j - g_k = d} sum g_j conj(v_k).
// One workgroup per (node, structure), 256 threads; thread t accumulates row
// t >> 2, columns (t & 3) + 4 e.
__global__ __launch_bounds__(256) void grad_assemble_kernel(GradArgs a) {
  __shared__ double2 vs[16][NP], gsh[16][NP];
  __shared__ double2 C[NP][NP + 1];
  const StructDev S = a.structs[blockIdx.y];
  const int n = blockIdx.x;
  if (S.n_beams > NP || n >= S.n_nodes) return;
  const int tid = threadIdx.x;
  const int res = n % a.nps;
  const int i0 = n / a.nps;
  // contributing (slice, stage) of node n
  int ci[2], cr[2], nc = 0;
  for (int t = 0; t < a.n_contrib[res]; ++t) {
    const int ii = i0 + a.contrib_di[res][t];
    if (ii >= 0 && ii < S.n_slices + a.last_extra) {
      ci[nc] = ii;
      cr[nc] = a.contrib_r[res][t];
      ++nc;
    }
  }
  // C = G^T conj(V) over t = (angle, contribution), a complex 64 x 64 x T
  // product on FP64 MFMA in the 3-real-product form: wave w owns rows
  // 16 w .. +15 and all 4 column tiles; chunks of 16 t through LDS (rows of
  // a short last chunk are zero).
  const int lane = tid & 63, w = tid >> 6;
  typedef double g4 __attribute__((ext_vector_type(4)));
  g4 p1[4], p2[4], p3[4];
#pragma unroll
  for (int jt = 0; jt < 4; ++jt) p1[jt] = p2[jt] = p3[jt] = g4{0, 0, 0, 0};
  const int total = S.n_angles * nc;
  for (int t0 = 0; t0 < total; t0 += 16) {
    const int cnt = min(16, total - t0);
    for (int e = tid; e < 16 * NP; e += 256) {
      const int tt = e / NP, jj = e % NP;
      double2 vv = make_double2(0.0, 0.0), gg = vv;
      if (tt < cnt) {
        const int t = t0 + tt;
        const int pr = S.pair_off + t / nc, c = t % nc;
        const double2* src = a.gbuf + (long long)pr * a.g_pair_stride + ((long long)ci[c] * a.stages + cr[c]) * 2 * NP;
        vv = src[jj];
        gg = src[NP + jj];
      }
      vs[tt][jj] = vv;
      gsh[tt][jj] = gg;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int tk = 4 * q + (lane >> 4);
      const double2 g = gsh[tk][16 * w + (lane & 15)];   // A[j][t] = g_t[j]
      const double gs = g.x + g.y;
#pragma unroll
      for (int jt = 0; jt < 4; ++jt) {
        const double2 v = vs[tk][16 * jt + (lane & 15)];  // B[t][k] = conj(v_t[k])
        p1[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(g.x, v.x, p1[jt], 0, 0, 0);
        p2[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(g.y, -v.y, p2[jt], 0, 0, 0);
        p3[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(gs, v.x - v.y, p3[jt], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int jt = 0; jt < 4; ++jt)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      C[16 * w + 4 * v + (lane >> 4)][16 * jt + (lane & 15)] =
          make_double2(p1[jt][v] - p2[jt][v], p3[jt][v] - p1[jt][v] - p2[jt][v]);
  __syncthreads();
  const int* bp = a.bin_ptr + S.bin_ptr_off;
  const int* bj = a.bin_jk + S.bin_jk_off;
  double2* out = a.dU + S.table_off + (long long)n * S.box;
  for (int d = tid; d < S.box; d += 256) {
    double2 v = make_double2(0.0, 0.0);
    for (int t = bp[d]; t < bp[d + 1]; ++t) {
      const int jk = bj[t];
      v = cadd(v, C[jk / NP][jk % NP]);
    }
    out[d] = v;
  }
}

// The same for structures with 64 < N <= 128 (stage buffer and bins of
// width NL): one workgroup of 8 waves per (node, structure); wave w owns rows
// 16 w .. +15 of C and all 8 column tiles.  C is binned one half of its rows
// at a time through LDS (the half shares the LDS with the chunk buffers),
// each table entry summing the first half's (j, k) in bin order, then the
// second's.
__global__ __launch_bounds__(512) void grad_assemble_wide_kernel(GradArgs a) {
  union GLds {
    struct {
      double2 vs[16][NL], gsh[16][NL];
    } in;
    double2 C[64][NL + 1];
  };
  __shared__ GLds sm;
  const StructDev S = a.structs[blockIdx.y];
  const int n = blockIdx.x;
  if (S.n_beams <= NP || S.n_beams > NL || n >= S.n_nodes) return;
  const int tid = threadIdx.x;
  const int res = n % a.nps;
  const int i0 = n / a.nps;
  int ci[2], cr[2], nc = 0;
  for (int t = 0; t < a.n_contrib[res]; ++t) {
    const int ii = i0 + a.contrib_di[res][t];
    if (ii >= 0 && ii < S.n_slices) {
      ci[nc] = ii;
      cr[nc] = a.contrib_r[res][t];
      ++nc;
    }
  }
  const int lane = tid & 63, w = tid >> 6;
  typedef double g4 __attribute__((ext_vector_type(4)));
  g4 p1[8], p2[8], p3[8];
#pragma unroll
  for (int jt = 0; jt < 8; ++jt) p1[jt] = p2[jt] = p3[jt] = g4{0, 0, 0, 0};
  const int total = S.n_angles * nc;
  for (int t0 = 0; t0 < total; t0 += 16) {
    const int cnt = min(16, total - t0);
    for (int e = tid; e < 16 * NL; e += 512) {
      const int tt = e / NL, jj = e % NL;
      double2 vv = make_double2(0.0, 0.0), gg = vv;
      if (tt < cnt) {
        const int t = t0 + tt;
        const int pr = S.pair_off + t / nc, c = t % nc;
        const double2* src = a.gbuf + (long long)pr * a.g_pair_stride + ((long long)ci[c] * a.stages + cr[c]) * 2 * NL;
        vv = src[jj];
        gg = src[NL + jj];
      }
      sm.in.vs[tt][jj] = vv;
      sm.in.gsh[tt][jj] = gg;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int tk = 4 * q + (lane >> 4);
      const double2 g = sm.in.gsh[tk][16 * w + (lane & 15)];   // A[j][t] = g_t[j]
      const double gs = g.x + g.y;
#pragma unroll
      for (int jt = 0; jt < 8; ++jt) {
        const double2 v = sm.in.vs[tk][16 * jt + (lane & 15)];  // B[t][k] = conj(v_t[k])
        p1[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(g.x, v.x, p1[jt], 0, 0, 0);
        p2[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(g.y, -v.y, p2[jt], 0, 0, 0);
        p3[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(gs, v.x - v.y, p3[jt], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  const int* bp = a.bin_ptr + S.bin_ptr_off;
  const int* bj = a.bin_jk + S.bin_jk_off;
  constexpr int DPT = (MAXBOXL + 511) / 512;  // table entries per thread
  double2 acc[DPT];
#pragma unroll
  for (int u = 0; u < DPT; ++u) acc[u] = make_double2(0.0, 0.0);
#pragma unroll 1
  for (int hv = 0; hv < 2; ++hv) {
    if ((w >> 2) == hv) {
#pragma unroll
      for (int jt = 0; jt < 8; ++jt)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          sm.C[16 * (w & 3) + 4 * v + (lane >> 4)][16 * jt + (lane & 15)] =
              make_double2(p1[jt][v] - p2[jt][v], p3[jt][v] - p1[jt][v] - p2[jt][v]);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < DPT; ++u) {
      const int d = tid + 512 * u;
      if (d < S.box) {
        for (int t = bp[d]; t < bp[d + 1]; ++t) {
          const int jk = bj[t], jr = jk / NL;
          if ((jr >> 6) == hv) acc[u] = cadd(acc[u], sm.C[jr - 64 * hv][jk % NL]);
        }
      }
    }
    __syncthreads();
  }
  double2* out = a.dU + S.table_off + (long long)n * S.box;
#pragma unroll
  for (int u = 0; u < DPT; ++u) {
    const int d = tid + 512 * u;
    if (d < S.box) out[d] = acc[u];
  }
}

// The same for structures with 128 < N <= 256 (stage buffer and bins of
// width NX): the 256 x 256 sum is formed in eight blocks of 128 rows x 64
// columns (one pass over the node's stage entries each; wave w owns rows
// 16 w .. +15 of the block) and each block is binned through LDS before the
// next, every table entry summing the blocks in order and, in each, its
// (j, k) in bin order.
__global__ __launch_bounds__(512) void grad_assemble_xl_kernel(GradArgs a) {
  union GLds {
    struct {
      double2 vs[16][64], gsh[16][128];
    } in;
    double2 C[128][65];
  };
  __shared__ GLds sm;
  const StructDev S = a.structs[blockIdx.y];
  const int n = blockIdx.x;
  if (S.n_beams <= NL || n >= S.n_nodes) return;
  const int tid = threadIdx.x;
  const int res = n % a.nps;
  const int i0 = n / a.nps;
  int ci[2], cr[2], nc = 0;
  for (int t = 0; t < a.n_contrib[res]; ++t) {
    const int ii = i0 + a.contrib_di[res][t];
    if (ii >= 0 && ii < S.n_slices + a.last_extra) {
      ci[nc] = ii;
      cr[nc] = a.contrib_r[res][t];
      ++nc;
    }
  }
  const int lane = tid & 63, w = tid >> 6;
  typedef double g4 __attribute__((ext_vector_type(4)));
  const int* bp = a.bin_ptr + S.bin_ptr_off;
  const int* bj = a.bin_jk + S.bin_jk_off;
  constexpr int DPT = (MAXBOXX + 511) / 512;  // table entries per thread
  double2 acc[DPT];
#pragma unroll
  for (int u = 0; u < DPT; ++u) acc[u] = make_double2(0.0, 0.0);
  const int total = S.n_angles * nc;
#pragma unroll 1
  for (int pass = 0; pass < 8; ++pass) {
    const int rh = pass >> 2, cq = pass & 3;  // rows 128 rh .., columns 64 cq ..
    g4 p1[4], p2[4], p3[4];
#pragma unroll
    for (int jt = 0; jt < 4; ++jt) p1[jt] = p2[jt] = p3[jt] = g4{0, 0, 0, 0};
    for (int t0 = 0; t0 < total; t0 += 16) {
      const int cnt = min(16, total - t0);
      for (int e = tid; e < 16 * 128; e += 512) {
        const int tt = e >> 7, jj = e & 127;
        double2 vv = make_double2(0.0, 0.0), gg = vv;
        if (tt < cnt) {
          const int t = t0 + tt;
          const int pr = S.pair_off + t / nc, c = t % nc;
          const double2* src =
              a.gbuf + (long long)pr * a.g_pair_stride + ((long long)ci[c] * a.stages + cr[c]) * 2 * NX;
          gg = src[NX + 128 * rh + jj];
          if (jj < 64) vv = src[64 * cq + jj];
        }
        sm.in.gsh[tt][jj] = gg;
        if (jj < 64) sm.in.vs[tt][jj] = vv;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int tk = 4 * q + (lane >> 4);
        const double2 g = sm.in.gsh[tk][16 * w + (lane & 15)];   // A[j][t] = g_t[j]
        const double gs = g.x + g.y;
#pragma unroll
        for (int jt = 0; jt < 4; ++jt) {
          const double2 v = sm.in.vs[tk][16 * jt + (lane & 15)];  // B[t][k] = conj(v_t[k])
          p1[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(g.x, v.x, p1[jt], 0, 0, 0);
          p2[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(g.y, -v.y, p2[jt], 0, 0, 0);
          p3[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(gs, v.x - v.y, p3[jt], 0, 0, 0);
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int jt = 0; jt < 4; ++jt)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        sm.C[16 * w + 4 * v + (lane >> 4)][16 * jt + (lane & 15)] =
            make_double2(p1[jt][v] - p2[jt][v], p3[jt][v] - p1[jt][v] - p2[jt][v]);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < DPT; ++u) {
      const int d = tid + 512 * u;
      if (d < S.box) {
        for (int t = bp[d]; t < bp[d + 1]; ++t) {
          const int jk = bj[t], jr = jk / NX, kc = jk % NX;
          if ((jr >> 7) == rh && (kc >> 6) == cq) acc[u] = cadd(acc[u], sm.C[jr - 128 * rh][kc - 64 * cq]);
        }
      }
    }
    __syncthreads();
  }
  double2* out = a.dU + S.table_off + (long long)n * S.box;
#pragma unroll
  for (int u = 0; u < DPT; ++u) {
    const int d = tid + 512 * u;
    if (d < S.box) out[d] = acc[u];
  }
}

hipError_t launch_backward(int stepper, int width, const BwdArgs& a, hipStream_t stream) {
  if (a.n_pairs < 1) return hipSuccess;
  const dim3 grid(2 * a.n_pairs);
  if (width == NX) {
    const dim3 block(BGeo<NX>::threads);
    if (stepper == 0)
      hipLaunchKernelGGL((backward_kernel<0, NX>), grid, block, 0, stream, a);
    else
      hipLaunchKernelGGL((backward_kernel<1, NX>), grid, block, 0, stream, a);
  } else if (width == NL) {
    const dim3 block(BGeo<NL>::threads);
    if (stepper == 0)
      hipLaunchKernelGGL((backward_kernel<0, NL>), grid, block, 0, stream, a);
    else
      hipLaunchKernelGGL((backward_kernel<1, NL>), grid, block, 0, stream, a);
  } else {
    const dim3 block(BGeo<NP>::threads);
    if (stepper == 0)
      hipLaunchKernelGGL((backward_kernel<0, NP>), grid, block, 0, stream, a);
    else if (stepper == 1)
      hipLaunchKernelGGL((backward_kernel<1, NP>), grid, block, 0, stream, a);
    else
      hipLaunchKernelGGL((backward_kernel<2, NP>), grid, block, 0, stream, a);
  }
  return hipGetLastError();
}

hipError_t launch_grad_assemble(const GradArgs& a, int n_struct, int max_nodes, bool narrow, bool wide, bool xl,
                                hipStream_t stream) {
  if (narrow) hipLaunchKernelGGL(grad_assemble_kernel, dim3(max_nodes, n_struct), dim3(256), 0, stream, a);
  if (wide) hipLaunchKernelGGL(grad_assemble_wide_kernel, dim3(max_nodes, n_struct), dim3(512), 0, stream, a);
  if (xl) hipLaunchKernelGGL(grad_assemble_xl_kernel, dim3(max_nodes, n_struct), dim3(512), 0, stream, a);
  return hipGetLastError();
}

}  // namespace rheed
