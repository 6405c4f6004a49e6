// Forward propagation for 256 < N <= 576 beams on gfx950 (part of the
// translation unit rheed_forward_all.hip, after rheed_forward_xl.hip, whose
// elimination, replay, reflection and group barrier it instantiates for its
// width).  This is the size of the paper's single-angle case (Sec. 4, the
// n = 521 data set), where batching over angles has nothing to batch: every
// pair runs in a group launch, its 16-column blocks spread over up to
// ceil(N / 16) workgroups.
//
// At NXX = 576 a column block's stage input (576 x 16 complex, 144 KB) no
// longer fits in LDS beside a node table, and the registers of a thread
// cannot hold its share of c, c' and the new state as they do for N <= 256.
// So a stage runs as:
//   * the stage input X_r = c + h c_r c' - h^2 sum_m (A^2)_{rm} G_m of the
//     block is formed XKC rows at a time into LDS (and into the workgroup's
//     memory, for the Gamma^2 X_r term), from c, c' and the earlier stage
//     products in memory;
//   * after each chunk every wave adds that chunk's k-range to the MFMA
//     accumulators of its row tiles (tiles w, w + 8, ..., up to five per
//     wave, each the 3-real-product form on v_mfma_f64_16x16x4f64 with the
//     node table gathered from LDS);
//   * G_r = U X_r + Gamma^2 X_r goes to memory; after the last stage each
//     thread forms the new c and c' of its tile entries from c, c' and the
//     stored stage products (summed in stage order) and adds their moduli to
//     the row sums of the badness.
// Everything after the slice (the Gershgorin / Varah decision, the
// transformation of Sec. 3.2 by a column elimination spread over the group
// in blocks of 16 steps and its replay on P, the reflection solve) is the
// N <= 256 group code at this width.

namespace rheed {
namespace {

constexpr int XXTP = (NXX / 16 + XW - 1) / XW;  // row tiles per wave (5)
constexpr int XKC = 128;                        // rows of the stage input per LDS chunk
constexpr int XXST = 7;                         // stage products kept per block (RK6)
constexpr int XXEM = 2;                         // rows per wave of an elimination block (2 x 9 per lane in registers)
constexpr int XXFR = 6;                         // multiplier rows a replay stages in LDS
constexpr int XXB = XKC * XCB > XXFR * NXX ? XKC * XCB : XXFR * NXX;  // entries of the shared buffer

static_assert(XXST * NXX * XCB * 16LL + NXX * XCB * 16LL <= XXG_STAGE_BYTES, "stage buffer of a workgroup");

struct XXLds {
  double2 xb[XXB];                  // a chunk of the stage input; the pivot rows of the eliminations;
                                    // the multiplier rows of a replay
  double2 tb[1][MAXBOXXX + 1];      // node table of the current stage; entry `box` stays 0
  int off[NXX];                     // h_k (2 kd + 1) + k_k of beam k
  int bhk[NXX][2];
  double g2s[NXX];                  // Gamma_j^2, 0 on padding
  double rdg[NXX], rof[NXX];        // per row: |q_ii| and sum_{j != i} |q_ij| over j < N
  int pcrec[NXX];                   // pivot column of every elimination step
  int pos[NXX];                     // pivot step of every column in the last elimination
  double2 xv[NXX];                  // first column of the inverse in the reflection
  unsigned long long bnorm_bits;
  unsigned long long xnorm_bits;
  int flag_singular;
  int bad;
  int sync_fail;
};
static_assert(XKC * XCB >= 2 * NXX, "the eliminations keep two pivot rows in the stage-input buffer");

__shared__ XXLds xxl_lds;

// One slice for the column blocks cb0, cb0 + cbs, ... that hold columns < N
// (see the head of this file); s.rdg / s.rof get those blocks' share of the
// row sums.  gm: [XXST][NXX][XCB] stage products, then the block's stage
// input [NXX][XCB].
template <int STEPPER>
__device__ __noinline__ void xxl_slice(double2* __restrict__ cg, double2* __restrict__ dg, double2* __restrict__ gm,
                                       const double2* __restrict__ Us, int nb, int box, double h, int N,
                                       const int (&base)[XXTP], int cb0, int cbs) {
  using T = LTab<STEPPER>;
  static_assert(T::stages <= XXST, "stage products of a block");
  XXLds& s = xxl_lds;
  const int tid = threadIdx.x, lane = tid & 63;
  // wave-uniform values in scalar registers, so that the tile tests below are scalar branches
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int n = __builtin_amdgcn_readfirstlane(N);
  const double hh = h * h;
  const int ncb = (n + XCB - 1) / XCB;
  const int ntile = (n + 15) / 16;
  double2* __restrict__ xg = gm + (long long)XXST * NXX * XCB;
  int tag = -1;  // node in the table slot (the same in every thread)
  __syncthreads();  // every wave has read the previous slice's row sums before they are cleared
  for (int j = tid; j < NXX; j += XT) {
    s.rdg[j] = 0.0;
    s.rof[j] = 0.0;
  }
#pragma unroll 1
  for (int cb = cb0; cb < ncb; cb += cbs) {
    const int col = XCB * cb + (lane & 15);  // this lane's column in the MFMA output layout
#pragma unroll 1
    for (int r = 0; r < T::stages; ++r) {
      const int nn = nb + T::node(r);
      if (tag != nn) {  // the previous stage's products have all read the slot (barrier at its end)
        for (int e = tid; e < box; e += XT) s.tb[0][e] = Us[(long long)nn * box + e];
        tag = nn;
      }
      const double hc = h * T::c(r);
      d4 p1[XXTP], p2[XXTP], p3[XXTP];
#pragma unroll
      for (int j = 0; j < XXTP; ++j) p1[j] = p2[j] = p3[j] = d4{0, 0, 0, 0};
#pragma unroll 1
      for (int k0 = 0; k0 < n; k0 += XKC) {
        __syncthreads();  // the previous chunk's products have read xb; the table is loaded
        // rows k0 .. k0 + XKC - 1 of X_r (rows >= N are zero: they meet zero entries of U)
        for (int e = tid; e < XKC * XCB; e += XT) {
          const int row = k0 + e / XCB, cl = e & (XCB - 1);
          double2 x = make_double2(0.0, 0.0);
          if (row < N) {
            const long long ix = (long long)row * NXX + XCB * cb + cl;
            const double2 c = gld(&cg[ix]), d = gld(&dg[ix]);
            double xr = c.x + hc * d.x, xi = c.y + hc * d.y;
#pragma unroll
            for (int m = 0; m < 6; ++m) {
              if (m < r && T::a2(r, m) != 0.0) {
                const double2 g = gld(&gm[((long long)m * NXX + row) * XCB + cl]);
                xr -= hh * T::a2(r, m) * g.x;
                xi -= hh * T::a2(r, m) * g.y;
              }
            }
            x = make_double2(xr, xi);
            gst(&xg[(long long)row * XCB + cl], x);
          }
          s.xb[e] = x;
        }
        __syncthreads();
        const int kr = n - k0 < XKC ? n - k0 : XKC;
        const int nq = (kr + 3) / 4;  // k-steps of 4 up to N (k < 4 ceil(N / 4) <= NXX)
        const double2* __restrict__ tsl = s.tb[0];
#pragma unroll 2
        for (int q = 0; q < nq; ++q) {
          const int kl = 4 * q + (lane >> 4);
          const int k = k0 + kl;
          const double2 x = s.xb[kl * XCB + (lane & 15)];
          const int ok = s.off[k];
          const bool kin = k < N;
          const double xs = x.x + x.y;
#pragma unroll
          for (int j = 0; j < XXTP; ++j) {
            if (w + XW * j < ntile) {  // wave-uniform
              const int ra = 16 * (w + XW * j) + (lane & 15);
              const double2 u = tsl[(kin && ra < N) ? base[j] - ok : box];
              p1[j] = mfma(u.x, x.x, p1[j]);
              p2[j] = mfma(u.y, x.y, p2[j]);
              p3[j] = mfma(u.x + u.y, xs, p3[j]);
            }
          }
        }
      }
      // G_r of this wave's tiles; after the last stage the block's new c and c'
#pragma unroll
      for (int j = 0; j < XXTP; ++j) {
        if (w + XW * j < ntile) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = 16 * (w + XW * j) + 4 * v + (lane >> 4);
            const bool rin = row < N;
            double gr = 0.0, gi = 0.0;
            if (rin) {
              const double2 x = gld(&xg[(long long)row * XCB + (lane & 15)]);
              const double g2v = s.g2s[row];
              gr = p1[j][v] - p2[j][v] + g2v * x.x;
              gi = p3[j][v] - p1[j][v] - p2[j][v] + g2v * x.y;
            }
            if (r + 1 < T::stages) {
              if (rin) gst(&gm[((long long)r * NXX + row) * XCB + (lane & 15)], make_double2(gr, gi));
            } else {
              double pd = 0.0, po = 0.0;
              if (rin) {
                const long long ix = (long long)row * NXX + col;
                const double2 c = gld(&cg[ix]), d = gld(&dg[ix]);
                double cnr = c.x + h * d.x, cni = c.y + h * d.y, dnr = d.x, dni = d.y;
#pragma unroll
                for (int m = 0; m < T::stages; ++m) {
                  double2 g;
                  if (m + 1 < T::stages) {
                    if (T::ba(m) == 0.0 && T::b(m) == 0.0) continue;
                    g = gld(&gm[((long long)m * NXX + row) * XCB + (lane & 15)]);
                  } else {
                    g = make_double2(gr, gi);
                  }
                  if (T::ba(m) != 0.0) {
                    cnr -= hh * T::ba(m) * g.x;
                    cni -= hh * T::ba(m) * g.y;
                  }
                  dnr -= h * T::b(m) * g.x;
                  dni -= h * T::b(m) * g.y;
                }
                gst(&cg[ix], make_double2(cnr, cni));
                gst(&dg[ix], make_double2(dnr, dni));
                if (col < N) {
                  const double av = sqrt(cnr * cnr + cni * cni);
                  if (row == col) pd = av;
                  else po = av;
                }
              }
#pragma unroll
              for (int o = 1; o < 16; o <<= 1) {
                pd += __shfl_xor(pd, o, 64);
                po += __shfl_xor(po, o, 64);
              }
              if ((lane & 15) == 0 && rin) {
                s.rdg[row] += pd;
                s.rof[row] += po;
              }
            }
          }
        }
      }
      __syncthreads();  // G_r and X_r reach the next stage's input; xb and the table slot are reused
    }
  }
  __syncthreads();
}

struct XXCfg {
  static constexpr int NXT = NXX;
  static constexpr int XEMT = XXEM;
  static constexpr int IDXB = 10;
  static constexpr int TSLOTS = 1;
  // the others wait at a barrier while workgroup 0 records an elimination of
  // up to 576 steps: a longer (still bounded) wait than for N <= 256
  static constexpr long long SYNC_TICKS = 10 * XCH_TICKS;
  static constexpr int SYNC_SPIN = 10 * XCH_SPIN;
  static constexpr int FROWS = XXFR;  // multiplier rows a replay stages in the stage-input buffer
  static constexpr long long PAIR_C = XXG_C, PAIR_D = XXG_D, PAIR_F = XXG_F, PAIR_PIV = XXG_PIV;
  static constexpr long long PAIR_BYTES = XXG_PAIR_BYTES;
  static constexpr long long WG_PART = XXG_STAGE_BYTES;
  static constexpr long long WG_BYTES = XXG_WG_BYTES;
  static __device__ __forceinline__ XXLds& lds() { return xxl_lds; }
  using Base = int[XXTP];
  // table index of U_{ik} = u_{g_i - g_k} is base_i - off_k for the A-operand
  // rows of the wave's tiles (rows beyond NXX: tiles that do not exist)
  template <bool F32>
  static __device__ __forceinline__ void bases(Base& base, int hd, int kd, int w, int lane) {
    static_assert(!F32, "FP64 stage products only at this width");
    const int Wd = 2 * kd + 1;
#pragma unroll
    for (int j = 0; j < XXTP; ++j) {
      const int i = 16 * (w + XW * j) + (lane & 15);
      base[j] = i < NXX ? (xxl_lds.bhk[i][0] + hd) * Wd + (xxl_lds.bhk[i][1] + kd) : 0;
    }
  }
  template <int STEPPER>
  static __device__ __forceinline__ void slice(double2* cg, double2* dg, double2* gm, const double2* Us, int nb,
                                               int box, double h, int N, const Base& base, int cb0, int cbs) {
    xxl_slice<STEPPER>(cg, dg, gm, Us, nb, box, h, N, base, cb0, cbs);
  }
  using ElimCfg = XXCfg;
};

template <int STEPPER>
__global__ __launch_bounds__(XT, 1) void forward_xxl_group_kernel(LargeArgs A, XlGroup X) {
  const int pi = blockIdx.x / X.group, g = blockIdx.x - pi * X.group;
  const int p = A.f.pair_list ? A.f.pair_list[pi] : pi;
  xl_run_pair<XXCfg, STEPPER, true, false>(A, p, nullptr, X, pi, g);
}

}  // namespace

hipError_t launch_forward_xxl_group(int stepper, const LargeArgs& a, const XlGroup& x, hipStream_t stream) {
  if (a.f.n_pairs < 1) return hipSuccess;
  if (x.group < 1 || (stepper != 0 && stepper != 1) || a.f.ws) return hipErrorInvalidValue;
  hipLaunchKernelGGL(xl_group_reset_kernel, dim3(1), dim3(256), 0, stream, x.counters, a.f.n_pairs);
  LargeArgs aa = a;
  XlGroup xx = x;
  void* params[] = {&aa, &xx};
  const void* f = stepper == 0 ? reinterpret_cast<const void*>(&forward_xxl_group_kernel<0>)
                               : reinterpret_cast<const void*>(&forward_xxl_group_kernel<1>);
  return hipLaunchCooperativeKernel(f, dim3(a.f.n_pairs * x.group), dim3(XT), params, 0, stream);
}

int forward_xxl_group_max_workgroups(int device) {
  int coop = 0, cus = 0, p0 = 0, p1 = 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) != hipSuccess || !coop) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&p0, forward_xxl_group_kernel<0>, XT, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&p1, forward_xxl_group_kernel<1>, XT, 0) != hipSuccess)
    return 0;
  const int per = p0 < p1 ? p0 : p1;
  return cus * (per > 0 ? per : 0);
}

}  // namespace rheed
