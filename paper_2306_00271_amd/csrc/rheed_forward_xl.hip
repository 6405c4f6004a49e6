// Forward propagation for 128 < N <= 256 beams on gfx950 (part of the
// translation unit rheed_forward_all.hip, after rheed_forward_large.hip,
// whose tableaux and slot helpers it uses).
//
// The state Z = [c; c'] padded to NX = 256 beams (2 MB) lives in a slot of
// device memory owned by the workgroup running the pair, as for N <= 128.
// At this size the stage products, not the memory traffic, bound a slice
// (7 x 8 N^3 flop against a few MB of slot reads), so the design keeps as
// little as possible on chip:
//   * a slice is stepped in blocks of 16 columns (the RK right-hand side
//     acts on columns independently); wave w of the 8 owns rows
//     32 w .. 32 w + 31 of the block (two 16 x 16 tiles of
//     v_mfma_f64_16x16x4f64, which share each B operand);
//   * the stage input X_r of the block is in LDS, formed from c and c' read
//     back from the slot and the earlier stage products G_m, which go to the
//     slot as they are made (the Nystrom combination needs up to five of
//     them, more than the registers of two tiles hold);
//   * U_jk = u_{g_j - g_k} is gathered from the node table of the stage in
//     LDS, loaded per stage into one of two table slots (a row of up to
//     MAXBOXX entries), with gather offsets from per-beam indices in LDS;
//   * c <- c + h c' - h^2 sum (bA)_m G_m and c' <- c' - h sum b_m G_m build
//     up in registers and go back to the slot after the block's last stage.
// The Gershgorin / Varah estimate of cond(Q) decides the transformation
// Z <- Z Q^{-1} (Sec. 3.2) as for N <= 128.  The elimination of Q (column
// Gauss-Jordan with partial pivoting, recording its multipliers) does not
// hold Q on chip: rows are taken 16 at a time (2 per wave, 4 columns per
// lane: more rows per wave spill on every step), the column operations of
// all earlier steps are replayed on them from the recorded multipliers
// (staged through LDS 16 rows at a time), and the block's own steps are then
// eliminated and recorded (a left-looking order of the same operations).
// The rows of P are replayed the same way, 16 at a time, and written back
// in pivot order: P Q^{-1}.  The reflection eliminates Gamma Q - iP likewise
// and applies the recorded operations in reverse to a unit vector.
//
// The launch is a persistent grid of one workgroup per CU over the pairs;
// no workgroup waits for another.  RK steppers; a separate instance keeps
// the states the adjoint reads, padded to NX.
//
// For a batch too small to fill the device (down to one pair) the same
// phases run in a group launch: G cooperatively launched workgroups per pair
// share the pair's state in memory and step the column blocks cb = g,
// g + G, ... of every slice (the RK stages act on columns independently).
// Per slice they meet at one barrier to sum their row-sum partials (in the
// same order in every workgroup, so all take the same decision); at a
// transformation the elimination runs in blocks of 16 steps, workgroup 0
// recording a block and every workgroup applying it to the later row blocks
// it owns, and all then replay it on their 16-row blocks of P.  Workgroup 0
// alone solves the reflection.  Both launches have an instance that keeps the
// adjoint's states.

namespace rheed {
namespace {

constexpr int XW = 8;             // waves per workgroup
constexpr int XT = XW * 64;       // threads per workgroup
constexpr int XCB = 16;           // columns per block
constexpr int XS = NX / 64;       // columns per lane in the eliminations

struct XLds {
  double2 xb[NX * XCB];           // stage input of a column block; the pivot rows of the eliminations
  double2 tb[2][MAXBOXX + 1];     // node tables of two stages; entry `box` of each stays 0
  int off[NX];                    // h_k (2 kd + 1) + k_k of beam k (the gather offset of column k)
  int bhk[NX][2];
  double g2s[NX];                 // Gamma_j^2, 0 on padding
  double rdg[NX], rof[NX];        // per row: |q_ii| and sum_{j != i} |q_ij| over j < N
  int pcrec[NX];                  // pivot column of every elimination step
  int pos[NX];                    // pivot step of every column in the last elimination
  double2 xv[NX];                 // first column of the inverse in the reflection
  unsigned long long bnorm_bits;  // ||Gamma Q - iP||_inf and ||x||_inf of the reflection
  unsigned long long xnorm_bits;
  int flag_singular;
  int bad;
  int sync_fail;                  // group launch: a wait of this workgroup gave up
};

__shared__ XLds xl_lds;

// Loads node nn of the structure's tables into table slot sl.
__device__ __forceinline__ void xl_load_table(int sl, const double2* __restrict__ Us, long long nn, int box) {
  for (int e = threadIdx.x; e < box; e += XT) xl_lds.tb[sl][e] = Us[nn * box + e];
}

// Matrix-core step of a stage product: FP64, or with F32 the operands
// rounded to FP32 on v_mfma_f32_16x16x4f32 (the lower-precision evaluation;
// the A rows are then supplied in a_row<true> order, so that register v
// holds the same row as in FP64).
__device__ __forceinline__ d4 mma(double a, double b, d4 c) { return mfma(a, b, c); }
__device__ __forceinline__ f4 mma(double a, double b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32((float)a, (float)b, c, 0, 0, 0);
}
template <bool F32> struct XAcc { using T = d4; };
template <> struct XAcc<true> { using T = f4; };

// One slice of the RK step for the column blocks cb0, cb0 + cbs, ... that
// hold columns < N; s.rdg / s.rof get those blocks' share of the row sums.
// F32: the stage products U X in FP32 (everything else FP64).
template <int STEPPER, bool F32>
__device__ __noinline__ void xl_slice(double2* __restrict__ cg, double2* __restrict__ dg, double2* __restrict__ gm,
                                      const double2* __restrict__ Us, int nb, int box, double h, int N,
                                      const int (&base)[2], int cb0, int cbs) {
  using T = LTab<STEPPER>;
  XLds& s = xl_lds;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const double hh = h * h;
  const int ncb = (N + XCB - 1) / XCB;
  const int nq = (N + 3) / 4;  // k-steps of 4 up to N: rows of X beyond meet zero entries of U
  double g2[2][4];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) g2[t][v] = s.g2s[32 * w + 16 * t + 4 * v + (lane >> 4)];
  int tag0 = -1, tag1 = -1;  // node held by each table slot (the same in every thread)
  __syncthreads();  // every wave has read the previous slice's row sums (the badness) before they are cleared
  if (tid < NX) {
    s.rdg[tid] = 0.0;
    s.rof[tid] = 0.0;
  }
  __syncthreads();
#pragma unroll 1
  for (int cb = cb0; cb < ncb; cb += cbs) {
    const int col = XCB * cb + (lane & 15);
    double cnr[2][4], cni[2][4], dnr[2][4], dni[2][4];
    double2 c0[2][4], d0[2][4];  // the block's c and c' at the slice start, for every stage input
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 32 * w + 16 * t + 4 * v + (lane >> 4);
        const double2 c = gld(&cg[row * NX + col]), d = gld(&dg[row * NX + col]);
        c0[t][v] = c;
        d0[t][v] = d;
        cnr[t][v] = c.x + h * d.x;
        cni[t][v] = c.y + h * d.y;
        dnr[t][v] = d.x;
        dni[t][v] = d.y;
      }
#pragma unroll 1
    for (int r = 0; r < T::stages; ++r) {
      const int nn = nb + T::node(r);
      int sl;
      if (tag0 == nn) {
        sl = 0;
      } else if (tag1 == nn) {
        sl = 1;
      } else {  // load into the slot the previous stage did not use
        sl = (r > 0 && tag0 == nb + T::node(r - 1)) ? 1 : 0;
        xl_load_table(sl, Us, nn, box);
        if (sl == 0) tag0 = nn;
        else tag1 = nn;
      }
      // X_r = c + h c_r c' - h^2 sum_{m < r} (A^2)_{rm} G_m, this thread's elements
      const double hc = h * T::c(r);
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 32 * w + 16 * t + 4 * v + (lane >> 4);
          const double2 c = c0[t][v], d = d0[t][v];
          double xr = c.x + hc * d.x, xi = c.y + hc * d.y;
#pragma unroll
          for (int m = 0; m < 6; ++m) {
            if (m < r && T::a2(r, m) != 0.0) {
              const double2 g = gld(&gm[(m * NX + row) * XCB + (lane & 15)]);
              xr -= hh * T::a2(r, m) * g.x;
              xi -= hh * T::a2(r, m) * g.y;
            }
          }
          s.xb[row * XCB + (lane & 15)] = make_double2(xr, xi);
        }
      __syncthreads();
      // G_r = U X_r + Gamma^2 X_r on the two tiles (3-real-product form)
      const double2* __restrict__ tsl = s.tb[sl];
      typename XAcc<F32>::T p1[2], p2[2], p3[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) p1[t] = p2[t] = p3[t] = {0, 0, 0, 0};
      const int ra0 = 32 * w + a_row<F32>(lane & 15), ra1 = ra0 + 16;  // A-operand rows of the two tiles
#pragma unroll 2
      for (int q = 0; q < nq; ++q) {
        const int k = 4 * q + (lane >> 4);
        const double2 x = s.xb[k * XCB + (lane & 15)];
        const int ok = s.off[k];
        const bool kin = k < N;
        const double2 u0 = tsl[(kin && ra0 < N) ? base[0] - ok : box];
        const double2 u1 = tsl[(kin && ra1 < N) ? base[1] - ok : box];
        const double xs = x.x + x.y;
        p1[0] = mma(u0.x, x.x, p1[0]);
        p2[0] = mma(u0.y, x.y, p2[0]);
        p3[0] = mma(u0.x + u0.y, xs, p3[0]);
        p1[1] = mma(u1.x, x.x, p1[1]);
        p2[1] = mma(u1.y, x.y, p2[1]);
        p3[1] = mma(u1.x + u1.y, xs, p3[1]);
      }
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 32 * w + 16 * t + 4 * v + (lane >> 4);
          const double2 x = s.xb[row * XCB + (lane & 15)];
          const double a1 = p1[t][v], a2 = p2[t][v], a3 = p3[t][v];
          const double gr = a1 - a2 + g2[t][v] * x.x;
          const double gi = a3 - a1 - a2 + g2[t][v] * x.y;
          if (r + 1 < T::stages) gst(&gm[(r * NX + row) * XCB + (lane & 15)], make_double2(gr, gi));
          if (T::ba(r) != 0.0) {
            cnr[t][v] -= hh * T::ba(r) * gr;
            cni[t][v] -= hh * T::ba(r) * gi;
          }
          dnr[t][v] -= h * T::b(r) * gr;
          dni[t][v] -= h * T::b(r) * gi;
        }
      __syncthreads();  // xb and the table slots are reused by the next stage
    }
    // the stepped block back to the slot, and its share of the row sums of |c|
    double pdg[2][4], pof[2][4];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 32 * w + 16 * t + 4 * v + (lane >> 4);
        gst(&cg[row * NX + col], make_double2(cnr[t][v], cni[t][v]));
        gst(&dg[row * NX + col], make_double2(dnr[t][v], dni[t][v]));
        const double av = sqrt(cnr[t][v] * cnr[t][v] + cni[t][v] * cni[t][v]);
        const bool in = row < N && col < N;
        pdg[t][v] = (in && row == col) ? av : 0.0;
        pof[t][v] = (in && row != col) ? av : 0.0;
      }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
          pdg[t][v] += __shfl_xor(pdg[t][v], o, 64);
          pof[t][v] += __shfl_xor(pof[t][v], o, 64);
        }
    if ((lane & 15) == 0) {
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 32 * w + 16 * t + 4 * v + (lane >> 4);
          s.rdg[row] += pdg[t][v];
          s.rof[row] += pof[t][v];
        }
    }
  }
  __syncthreads();
}

// The phases after the stage products (badness, elimination, replay,
// reflection, group barrier) are shared with the kernel for wider
// structures; a width configuration gives them the padded beam count, the
// rows per wave of an elimination block, the LDS and the layout of a pair's
// memory.
struct XCfg {
  static constexpr int NXT = NX;
  static constexpr int XEMT = 2;  // rows per wave of an elimination or replay block (16-row blocks)
  static constexpr int IDXB = 8;        // bits of the column index in a pivot key
  static constexpr int TSLOTS = 2;      // node-table slots in LDS
  static constexpr long long SYNC_TICKS = XCH_TICKS;  // a group barrier's wait gives up after this
  static constexpr int SYNC_SPIN = XCH_SPIN;          // or after this many polls
  static constexpr int FROWS = XCB;                   // multiplier rows a replay stages in the stage-input buffer
  using ElimCfg = XCfg;                               // the one-workgroup eliminations (and the reflection's)
  static constexpr long long PAIR_C = XSLOT_C, PAIR_D = XSLOT_D, PAIR_F = XSLOT_F, PAIR_PIV = XSLOT_G;
  static constexpr long long PAIR_BYTES = XG_PAIR_BYTES;
  static constexpr long long WG_PART = XG_STAGE_BYTES;  // row-sum partials after the stage products
  static constexpr long long WG_BYTES = XG_WG_BYTES;
  static __device__ __forceinline__ XLds& lds() { return xl_lds; }
  using Base = int[2];
  // table index of U_{ik} = u_{g_i - g_k} is base_i - off_k for the A-operand
  // rows of the thread's two tiles
  template <bool F32>
  static __device__ __forceinline__ void bases(Base& base, int hd, int kd, int w, int lane) {
    const int Wd = 2 * kd + 1;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int i = 32 * w + 16 * t + a_row<F32>(lane & 15);
      base[t] = (xl_lds.bhk[i][0] + hd) * Wd + (xl_lds.bhk[i][1] + kd);
    }
  }
  // STEPPER: bits 0-2 the method, bit 3 the FP32 stage products
  template <int STEPPER>
  static __device__ __forceinline__ void slice(double2* cg, double2* dg, double2* gm, const double2* Us, int nb,
                                               int box, double h, int N, const Base& base, int cb0, int cbs) {
    xl_slice<(STEPPER & 7), (STEPPER & F32_STAGES) != 0>(cg, dg, gm, Us, nb, box, h, N, base, cb0, cbs);
  }
};



// Rows m < R of z: column j <- column j - f_j column pc, pc = 64 HF + pl
// (the pivot column's quarter is wave-uniform, so it selects code).
template <int HF, int R, int XSN>
__device__ __forceinline__ void xl_col_update(double2 (&z)[R][XSN], int pl, const double2 (&f)[XSN]) {
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const double2 zp = make_double2(readlane_f64(z[m][HF].x, pl), readlane_f64(z[m][HF].y, pl));
#pragma unroll
    for (int q = 0; q < XSN; ++q) {
      z[m][q].x = fma(-f[q].x, zp.x, z[m][q].x);
      z[m][q].x = fma(f[q].y, zp.y, z[m][q].x);
      z[m][q].y = fma(-f[q].x, zp.y, z[m][q].y);
      z[m][q].y = fma(-f[q].y, zp.x, z[m][q].y);
    }
    if ((m & 1) == 1) __builtin_amdgcn_sched_barrier(0);
  }
}

template <int R, int XSN, int H>
__device__ __forceinline__ void xl_update_from(double2 (&z)[R][XSN], int hf, int pl, const double2 (&f)[XSN]) {
  if constexpr (H + 1 == XSN) {
    xl_col_update<H, R, XSN>(z, pl, f);
  } else {
    if (hf == H) xl_col_update<H, R, XSN>(z, pl, f);
    else xl_update_from<R, XSN, H + 1>(z, hf, pl, f);
  }
}

template <int R, int XSN>
__device__ __forceinline__ void xl_update(double2 (&z)[R][XSN], int pc, const double2 (&f)[XSN]) {
  const int hf = pc >> 6, pl = pc & 63;
  if constexpr (XSN == 4) {
    switch (hf) {
      case 0: xl_col_update<0, R, 4>(z, pl, f); break;
      case 1: xl_col_update<1, R, 4>(z, pl, f); break;
      case 2: xl_col_update<2, R, 4>(z, pl, f); break;
      default: xl_col_update<3, R, 4>(z, pl, f); break;
    }
  } else {
    xl_update_from<R, XSN, 0>(z, hf, pl, f);
  }
}

// The recorded column operations of steps [k0, k1) on the rows in z.  The
// multiplier rows are staged through the stage-input buffer (free during
// every replay) C::FROWS at a time by the whole workgroup, with direct
// global-to-LDS loads all in flight at once, so each chunk costs one memory
// latency instead of one per step; every wave calls it with the same k0 and
// k1.
template <class C, int R>
__device__ __forceinline__ void xl_replay(double2 (&z)[R][C::NXT / 64], int k0, int k1, int lane,
                                          const double2* __restrict__ frec) {
  constexpr int NXT = C::NXT, XST = NXT / 64, FR = C::FROWS;
  double2* fb = C::lds().xb;
  const int wu = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll 1
  for (int kc = k0; kc < k1; kc += FR) {
    const int kn = k1 - kc < FR ? k1 - kc : FR;
    __syncthreads();  // the previous chunk is consumed; the buffer's other users are done
    // 64-entry pieces of the kn rows (NXT is a multiple of 64), one 16-byte load per lane
    for (int t = wu; t < kn * XST; t += XW)
      __builtin_amdgcn_global_load_lds((const void*)(frec + (long long)kc * NXT + 64 * t + lane),
                                       (__attribute__((address_space(3))) void*)(fb + 64 * t), 16, 0, 0);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
#pragma unroll 1
    for (int j = 0; j < kn; ++j) {
      double2 f[XST];
#pragma unroll
      for (int q = 0; q < XST; ++q) f[q] = fb[j * NXT + 64 * q + lane];
      xl_update<R, XST>(z, __builtin_amdgcn_readfirstlane(C::lds().pcrec[kc + j]), f);
    }
  }
}

// Steps k0 .. k1 - 1 of a recording elimination, on the rows of the block
// that starts at row k0 (rows k0 + w + XW m of it in wave w, in z, each
// carrying every earlier step): step k picks, among the unused columns < n
// (um, the same in every wave), the one with the largest |A_kj| (key: the
// upper 32 bits of |A_kj|^2 with the low C::IDXB bits replaced by the
// complement of j, so near-ties go to the smaller index), records
// f_j = A_kj / A_k,pc (f_pc = 1 - 1 / A_k,pc) in frec and its pivot column in
// s.pcrec, and subtracts f_j column pc from every column j of the block's
// rows.  Row k + 1 reaches the other waves through LDS.
template <class C>
__device__ __forceinline__ void xl_record_steps(double2 (&z)[C::XEMT][C::NXT / 64],
                                                unsigned long long (&um)[C::NXT / 64], int k0, int k1, int n,
                                                double2* __restrict__ frec) {
  constexpr int NXT = C::NXT, XST = NXT / 64, XEMT = C::XEMT;
  constexpr unsigned IDXM = (1u << C::IDXB) - 1u;
  static_assert(NXT <= (1 << C::IDXB), "pivot keys hold every column index");
  auto& s = C::lds();
  const int tid = threadIdx.x, lane = tid & 63;
  const int wu = __builtin_amdgcn_readfirstlane(tid >> 6);
  double2* rowbuf = s.xb;
  __syncthreads();  // rowbuf aliases the stage buffer and the previous block's last row
  if (wu == 0) {
#pragma unroll
    for (int q = 0; q < XST; ++q) rowbuf[64 * q + lane] = z[0][q];
  }
#pragma unroll 1
  for (int k = k0; k < k1; ++k) {
    const int slot = k & 1;
    __syncthreads();
    double2 v[XST];
    unsigned key = 0;
#pragma unroll
    for (int q = 0; q < XST; ++q) {
      v[q] = rowbuf[slot * NXT + 64 * q + lane];
      const int c = 64 * q + lane;
      if (!((um[q] >> lane) & 1ull) && c < n) {
        const double m2 = v[q].x * v[q].x + v[q].y * v[q].y;
        const unsigned kq =
            ((unsigned)(((unsigned long long)__double_as_longlong(m2)) >> 32) & ~IDXM) | (IDXM - (unsigned)c);
        key = kq > key ? kq : key;
      }
    }
    key = wave_max_u32(key);
    if ((key >> C::IDXB) == 0 && tid == 0) s.flag_singular = 1;
    const int pc = (int)(IDXM - (key & IDXM));
    const int hf = pc >> 6, pl = pc & 63;
#pragma unroll
    for (int q = 0; q < XST; ++q)
      if (q == hf) um[q] |= 1ull << pl;
    double2 vs = v[0];
#pragma unroll
    for (int q = 1; q < XST; ++q)
      if (q == hf) vs = v[q];
    const double2 piv = make_double2(readlane_f64(vs.x, pl), readlane_f64(vs.y, pl));
    const double inv = 1.0 / (piv.x * piv.x + piv.y * piv.y);
    const double2 ip = make_double2(piv.x * inv, -piv.y * inv);
    double2 f[XST];
#pragma unroll
    for (int q = 0; q < XST; ++q) {
      f[q] = make_double2(v[q].x * ip.x - v[q].y * ip.y, v[q].x * ip.y + v[q].y * ip.x);
      if (q == hf && lane == pl) f[q] = make_double2(1.0 - ip.x, -ip.y);
    }
    if (wu == 0) {
#pragma unroll
      for (int q = 0; q < XST; ++q) gst(&frec[k * NXT + 64 * q + lane], f[q]);
      if (lane == 0) s.pcrec[k] = pc;
    }
    xl_update<XEMT, XST>(z, pc, f);
    // row k + 1 of this block: wave (k + 1 - k0) % XW, register (k + 1 - k0) / XW
    const int nx = k + 1 - k0;
    if (k + 1 < k1 && wu == (nx & (XW - 1))) {
      const int mr = nx / XW;
#pragma unroll
      for (int m = 0; m < XEMT; ++m)
        if (m == mr) {
#pragma unroll
          for (int q = 0; q < XST; ++q) rowbuf[(slot ^ 1) * NXT + 64 * q + lane] = z[m][q];
        }
    }
  }
}

// Recording elimination of the n x n leading block of Q = c (which = 0) or
// of Gamma Q - iP (which = 1), XW * C::XEMT rows at a time (a left-looking
// order): the steps of earlier blocks are replayed on a block's rows, then
// its own steps are taken (xl_record_steps).  s.pos gets the step at which
// each column was the pivot (its own index for columns >= n).
template <class C>
__device__ __noinline__ void xl_elim_record(const double2* __restrict__ cg, const double2* __restrict__ dg,
                                            double2* __restrict__ frec, int N, int which) {
  constexpr int NXT = C::NXT, XST = NXT / 64, XEMT = C::XEMT, XEBT = XW * XEMT;
  auto& s = C::lds();
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int n = __builtin_amdgcn_readfirstlane(N);
  const int wu = __builtin_amdgcn_readfirstlane(w);
  const bool refl = __builtin_amdgcn_readfirstlane(which) != 0;
  unsigned long long um[XST];  // used columns (the same in every wave)
#pragma unroll
  for (int q = 0; q < XST; ++q) um[q] = 0;
#pragma unroll 1
  for (int k0 = 0; k0 < n; k0 += XEBT) {
    double2 z[XEMT][XST];
#pragma unroll
    for (int m = 0; m < XEMT; ++m) {
      const int row = k0 + wu + XW * m;
      double gr = 0.0, gi = 0.0;
      if (refl && row < n) {
        const double g2v = s.g2s[row];
        gr = g2v >= 0.0 ? sqrt(g2v) : 0.0;
        gi = g2v >= 0.0 ? 0.0 : -sqrt(-g2v);
      }
#pragma unroll
      for (int q = 0; q < XST; ++q) {
        const int c = 64 * q + lane;
        double2 v = make_double2(0.0, 0.0);
        if (row < n) {
          const double2 cv = gld(&cg[row * NXT + c]);
          if (refl) {
            const double2 pv = gld(&dg[row * NXT + c]);
            v = make_double2(gr * cv.x - gi * cv.y + pv.y, gr * cv.y + gi * cv.x - pv.x);
          } else {
            v = cv;
          }
        }
        z[m][q] = v;
      }
    }
    __syncthreads();  // the previous block's last multipliers are stored
    xl_replay<C, XEMT>(z, 0, k0, lane, frec);
    xl_record_steps<C>(z, um, k0, n < k0 + XEBT ? n : k0 + XEBT, n, frec);
  }
  // the multipliers and pivot list are read back by this workgroup only
  __syncthreads();
  for (int j = tid; j < NXT; j += XT) s.pos[j] = j;
  __syncthreads();
  for (int j = tid; j < n; j += XT) s.pos[s.pcrec[j]] = j;
  __syncthreads();
}

// P <- P Q^{-1} after xl_elim_record(which = 0): the recorded operations on
// the rows of P, 64 at a time (row blocks b0, b0 + bs, ...), each column put
// at its pivot step; c <- I on the same rows.
template <class C>
__device__ __noinline__ void xl_replay_p(double2* __restrict__ cg, double2* __restrict__ dg,
                                         const double2* __restrict__ frec, int N, int b0, int bs) {
  constexpr int NXT = C::NXT, XST = NXT / 64, XEMT = C::XEMT, XEBT = XW * XEMT;
  auto& s = C::lds();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int n = __builtin_amdgcn_readfirstlane(N);
  int pq[XST];
#pragma unroll
  for (int q = 0; q < XST; ++q) pq[q] = s.pos[64 * q + lane];
  // rows >= n are zero rows of P and unit rows of c, which the
  // transformation leaves as they are
#pragma unroll 1
  for (int r0 = XEBT * b0; r0 < n; r0 += XEBT * bs) {
    double2 z[XEMT][XST];
#pragma unroll
    for (int m = 0; m < XEMT; ++m)
#pragma unroll
      for (int q = 0; q < XST; ++q) z[m][q] = gld(&dg[(r0 + w + XW * m) * NXT + 64 * q + lane]);
    xl_replay<C, XEMT>(z, 0, n, lane, frec);
#pragma unroll
    for (int m = 0; m < XEMT; ++m) {
      const int row = r0 + w + XW * m;
#pragma unroll
      for (int q = 0; q < XST; ++q) {
        gst(&dg[row * NXT + pq[q]], z[m][q]);
        gst(&cg[row * NXT + 64 * q + lane], make_double2(row == 64 * q + lane ? 1.0 : 0.0, 0.0));
      }
    }
  }
  __syncthreads();
}

// Bounded wait of a workgroup until *word >= target (thread 0 polls, then
// acquires).  It gives up after C::SYNC_SPIN polls or C::SYNC_TICKS of the
// constant-rate clock (about 20 ms for N <= 256, 200 ms for the wider kernel,
// whose eliminations are longer), sets s.sync_fail and the pair's failure
// word, and returns at once after an earlier give-up.
template <class C>
__device__ __forceinline__ void xl_wait_geq(const unsigned* word, unsigned target, unsigned* fail_word) {
  if (threadIdx.x == 0) {
    if (!C::lds().sync_fail) {
      const long long t0 = wall_clock64();
      int it = 0;
      while (__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (++it > C::SYNC_SPIN || wall_clock64() - t0 > C::SYNC_TICKS) {
          C::lds().sync_fail = 1;
          __hip_atomic_store(fail_word, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// Barrier of the G workgroups of one pair in a group launch: each raises the
// pair's counter (an agent-scope release, so its stores are written back
// first) and waits until all have reached `target` (G times the barriers so
// far), then acquires (xl_wait_geq: the wait is bounded, and a workgroup
// whose wait gave up stops waiting from then on).
template <class C>
__device__ __forceinline__ void xl_group_sync(unsigned* cnt, unsigned target, unsigned* fail_word) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's stores are issued and complete
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  xl_wait_geq<C>(cnt, target, fail_word);
}

// Publishes value in *word (one writer per word) once every wave's stores
// are complete: an agent-scope release, so the stores are written back first.
__device__ __forceinline__ void xl_publish(unsigned* word, unsigned value) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(word, value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// The transformation's elimination of Q (Sec. 3.2) spread over a pair's
// group of G >= 2 workgroups in blocks of XW * C::XEMT steps, as a pipeline.
// Row block bb belongs to workgroup 1 + bb mod (G - 1).  Workgroup 0 takes
// the blocks in turn: it waits until the owner of block b has applied the
// steps of block b - 2 to it, applies block b - 1's steps itself, records
// block b's steps (multipliers to frec, pivot columns to the pair's list)
// and publishes ctr[2] = e0 + b + 1.  Owner g, for each block b, waits for
// that word, applies block b's steps to its blocks >= b + 2, writes them back
// and publishes ctr[3 + g] = e0 + b + 1.  Every row meets the same column
// operations in the same order as in the one-workgroup elimination, so the
// multipliers are the same; c holds the partly eliminated rows meanwhile (the
// replay on P that follows sets it to I).  e0 counts the pair's earlier
// blocks, so the words only grow within a launch.

// Workgroup 0's part.
template <class C>
__device__ __noinline__ void xl_pipe_record(const double2* __restrict__ cg, double2* __restrict__ frec,
                                            int* __restrict__ pivg, int N, int G, unsigned* ctr, unsigned e0) {
  constexpr int NXT = C::NXT, XST = NXT / 64, XEMT = C::XEMT, XEBT = XW * XEMT;
  auto& s = C::lds();
  const int tid = threadIdx.x, lane = tid & 63;
  const int wu = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int n = __builtin_amdgcn_readfirstlane(N);
  const int gs = __builtin_amdgcn_readfirstlane(G);
  const int nb = (n + XEBT - 1) / XEBT;
  unsigned long long um[XST];  // used columns (the same in every wave)
#pragma unroll
  for (int q = 0; q < XST; ++q) um[q] = 0;
#pragma unroll 1
  for (int b = 0; b < nb; ++b) {
    const int k0 = XEBT * b, k1 = n < k0 + XEBT ? n : k0 + XEBT;
    if (b >= 2) xl_wait_geq<C>(&ctr[3 + 1 + b % (gs - 1)], e0 + b - 1, ctr + 1);
    double2 z[XEMT][XST];
#pragma unroll
    for (int m = 0; m < XEMT; ++m) {
      const int row = k0 + wu + XW * m;
#pragma unroll
      for (int q = 0; q < XST; ++q)
        z[m][q] = row < n ? gld(&cg[(long long)row * NXT + 64 * q + lane]) : make_double2(0.0, 0.0);
    }
    if (b >= 1) {
      __syncthreads();  // the previous block's last multipliers are stored
      xl_replay<C, XEMT>(z, k0 - XEBT, k0, lane, frec);
    }
    xl_record_steps<C>(z, um, k0, k1, n, frec);
    __syncthreads();
    for (int j = tid; j < k1 - k0; j += XT) pivg[k0 + j] = s.pcrec[k0 + j];
    xl_publish(&ctr[2], e0 + b + 1);
  }
}

// Owner g's part (1 <= g < G).
template <class C>
__device__ __noinline__ void xl_pipe_apply(double2* __restrict__ cg, const double2* __restrict__ frec,
                                           const int* __restrict__ pivg, int N, int g, int G, unsigned* ctr,
                                           unsigned e0) {
  constexpr int NXT = C::NXT, XST = NXT / 64, XEMT = C::XEMT, XEBT = XW * XEMT;
  auto& s = C::lds();
  const int tid = threadIdx.x, lane = tid & 63;
  const int wu = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int n = __builtin_amdgcn_readfirstlane(N);
  const int gu = __builtin_amdgcn_readfirstlane(g), go = __builtin_amdgcn_readfirstlane(G) - 1;
  const int nb = (n + XEBT - 1) / XEBT;
#pragma unroll 1
  for (int b = 0; b + 2 < nb; ++b) {
    const int k0 = XEBT * b, k1 = n < k0 + XEBT ? n : k0 + XEBT;
    xl_wait_geq<C>(&ctr[2], e0 + b + 1, ctr + 1);
    // the block's pivot columns (brought into range: after a failed wait the
    // list may be stale)
    for (int j = tid; j < k1 - k0; j += XT) s.pcrec[k0 + j] = (int)((unsigned)pivg[k0 + j] % (unsigned)NXT);
    __syncthreads();
#pragma unroll 1
    for (int bb = b + 2 + (((gu - 1) - (b + 2) % go) + go) % go; bb < nb; bb += go) {
      double2 z[XEMT][XST];
#pragma unroll
      for (int m = 0; m < XEMT; ++m) {
        const int row = XEBT * bb + wu + XW * m;
#pragma unroll
        for (int q = 0; q < XST; ++q)
          z[m][q] = row < n ? gld(&cg[(long long)row * NXT + 64 * q + lane]) : make_double2(0.0, 0.0);
      }
      xl_replay<C, XEMT>(z, k0, k1, lane, frec);
#pragma unroll
      for (int m = 0; m < XEMT; ++m) {
        const int row = XEBT * bb + wu + XW * m;
        if (row < n) {
#pragma unroll
          for (int q = 0; q < XST; ++q) gst(&cg[(long long)row * NXT + 64 * q + lane], z[m][q]);
        }
      }
    }
    xl_publish(&ctr[3 + gu], e0 + b + 1);
  }
}

// The group elimination (ends after a barrier, with frec and the pair's
// pivot list complete); a group of one runs the one-workgroup elimination.
template <class C>
__device__ __forceinline__ void xl_group_elim(double2* cg, const double2* dg, double2* frec, int* pivg, int N,
                                              int g, int G, unsigned* ctr, unsigned& nsync, unsigned& eblk) {
  constexpr int XEBT = XW * C::XEMT;
  if (G == 1) {
    xl_elim_record<typename C::ElimCfg>(cg, dg, frec, N, 0);
    for (int j = threadIdx.x; j < N; j += XT) pivg[j] = C::lds().pcrec[j];
  } else if (g == 0) {
    xl_pipe_record<C>(cg, frec, pivg, N, G, ctr, eblk);
  } else {
    xl_pipe_apply<C>(cg, frec, pivg, N, g, G, ctr, eblk);
  }
  eblk += (N + XEBT - 1) / XEBT;
  xl_group_sync<C>(ctr, G * ++nsync, ctr + 1);
}

// Q^{-1} (or B^{-1} of the reflection) after xl_elim_record: the recorded
// column operations replayed on the rows of I, XW * XCfg::XEMT at a time (row
// blocks b0, b0 + bs, ...), each column put at its pivot step as in
// xl_replay_p; rows to out (row major, stride NX; rows >= n stay unit rows).
__device__ __noinline__ void xl_replay_identity(double2* __restrict__ out, const double2* __restrict__ frec, int N,
                                                int b0, int bs) {
  constexpr int RM = XCfg::XEMT, RB = XW * RM;
  XLds& s = xl_lds;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int n = __builtin_amdgcn_readfirstlane(N);
  int pq[XS];
#pragma unroll
  for (int q = 0; q < XS; ++q) pq[q] = s.pos[64 * q + lane];
#pragma unroll 1
  for (int r0 = RB * b0; r0 < NX; r0 += RB * bs) {
    double2 z[RM][XS];
#pragma unroll
    for (int m = 0; m < RM; ++m)
#pragma unroll
      for (int q = 0; q < XS; ++q) z[m][q] = make_double2(r0 + w + XW * m == 64 * q + lane ? 1.0 : 0.0, 0.0);
    if (r0 < n) xl_replay<XCfg, RM>(z, 0, n, lane, frec);
#pragma unroll
    for (int m = 0; m < RM; ++m) {
      const int row = r0 + w + XW * m;
#pragma unroll
      for (int q = 0; q < XS; ++q) gst(&out[row * NX + pq[q]], z[m][q]);
    }
  }
}

// Copy of an NX x NX block of the slot (for the states the adjoint reads).
__device__ __forceinline__ void xl_copy(double2* __restrict__ dst, const double2* __restrict__ src) {
  for (int e = threadIdx.x; e < NX * NX; e += XT) gst(&dst[e], gld(&src[e]));
}

// The same for the 16-column blocks cb0, cb0 + cbs, ... of the NX / 16 (a
// workgroup's share of a state in a group launch: the blocks it steps).
__device__ __forceinline__ void xl_copy_cols(double2* __restrict__ dst, const double2* __restrict__ src, int cb0,
                                             int cbs) {
#pragma unroll 1
  for (int cb = cb0; cb < NX / XCB; cb += cbs)
    for (int e = threadIdx.x; e < NX * XCB; e += XT) {
      const int i = (e / XCB) * NX + XCB * cb + (e & (XCB - 1));
      gst(&dst[i], gld(&src[i]));
    }
}

// The same for the RB-row blocks b0, b0 + bs, ... of the NX / RB.
template <int RB>
__device__ __forceinline__ void xl_copy_rows(double2* __restrict__ dst, const double2* __restrict__ src, int b0,
                                             int bs) {
#pragma unroll 1
  for (int b = b0; b < NX / RB; b += bs)
    for (int e = threadIdx.x; e < RB * NX; e += XT) gst(&dst[RB * NX * b + e], gld(&src[RB * NX * b + e]));
}

// One pair.  GRP: workgroup g of the pair's G in a group launch (state,
// multipliers and pivot list in the pair's block of X.pair_mem, stage
// products and row-sum partials in the workgroup's block of X.wg_mem);
// otherwise the whole pair in this workgroup's slot.  SAVE: keep the states
// the adjoint reads, padded to NX: the state at the start of every
// ck.every-th slice and after the last, T = Q^{-1} and (ck.every > 1) R of
// every transformation, one decision byte per slice and B^{-1} of the
// reflection solve.  In a group launch each workgroup copies the column
// blocks of the states that it steps itself (no other workgroup writes them
// until the next barrier) and a share of the row blocks of T and R; the
// decision bytes and B^{-1} are workgroup 0's.
template <class C, int STEPPER, bool GRP, bool SAVE = false>
__device__ void xl_run_pair(const LargeArgs& A, int p, char* slot, const XlGroup& X, int pi, int g) {
  static_assert(!SAVE || C::NXT == NX, "states are kept for N <= 256");
  static_assert(GRP || C::NXT == NX, "the one-workgroup launch is for N <= 256");
  constexpr bool F32 = (STEPPER & F32_STAGES) != 0;  // FP32 stage products
  static_assert(!(F32 && SAVE), "the adjoint's states come from FP64 stages");
  using T = LTab<(STEPPER & 7)>;
  constexpr int NXT = C::NXT, XST = NXT / 64;
  const FwdArgs& a = A.f;
  auto& s = C::lds();
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int G = GRP ? X.group : 1;
  char* pm = GRP ? X.pair_mem + (long long)pi * C::PAIR_BYTES : slot;
  char* wm = GRP ? X.wg_mem + ((long long)pi * G + g) * C::WG_BYTES : slot + XSLOT_G;
  double2* __restrict__ cg = reinterpret_cast<double2*>(pm + C::PAIR_C);
  double2* __restrict__ dg = reinterpret_cast<double2*>(pm + C::PAIR_D);
  double2* __restrict__ frec = reinterpret_cast<double2*>(pm + C::PAIR_F);
  double2* __restrict__ gm = reinterpret_cast<double2*>(wm);
  int* pivg = reinterpret_cast<int*>(pm + C::PAIR_PIV);  // GRP: the pivot list of the last elimination
  unsigned* cnt = GRP ? X.counters + (long long)XG_CTR_WORDS * pi : nullptr;
  unsigned* failw = GRP ? cnt + 1 : nullptr;
  unsigned nsync = 0;  // group barriers so far
  unsigned eblk = 0;   // elimination blocks so far (the pipeline's progress words count them)
  char* pws = SAVE ? a.ws + (long long)p * a.ck.pair_stride : nullptr;
  constexpr long long MATB = (long long)NX * NX * sizeof(double2);
  const StructDev S = a.structs[a.pair_struct[p]];
  const int N = S.n_beams;
  const int L = S.n_slices;
  const double h = S.h;
  const double2* __restrict__ Us = a.U + S.table_off;
  const int Wd = 2 * S.kd + 1;

  for (int j = tid; j < NXT; j += XT) {
    const int hk0 = j < N ? a.beams[2 * (S.beam_off + j)] : 0;
    const int hk1 = j < N ? a.beams[2 * (S.beam_off + j) + 1] : 0;
    s.bhk[j][0] = hk0;
    s.bhk[j][1] = hk1;
    s.off[j] = hk0 * Wd + hk1;
  }
  if (tid == 0) {
    s.flag_singular = 0;
    s.bad = 0;
    s.sync_fail = 0;
    if constexpr (GRP) {
      // failure path for tests (rheed_plan_force_sync_failure): this
      // workgroup starts as if its first wait had given up
      if (a.xch_give_up == g) {
        s.sync_fail = 1;
        __hip_atomic_store(failw, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
  if (tid < C::TSLOTS) s.tb[tid][S.box] = make_double2(0.0, 0.0);
  __syncthreads();
  const double th0 = a.angles[2 * p], th1 = a.angles[2 * p + 1];
  for (int j = tid; j < NXT; j += XT) {
    // Gamma_j^2 = gamma^2 - |b0 + k_j|^2 (Sec. 2.1), b0 = gamma cos(theta0) (cos theta1, sin theta1)
    const double b0x = S.gamma * cos(th0) * cos(th1);
    const double b0y = S.gamma * cos(th0) * sin(th1);
    double arg = 0.0;
    if (j < N) {
      const double qx = b0x + s.bhk[j][0] * S.recip[0] + s.bhk[j][1] * S.recip[2];
      const double qy = b0y + s.bhk[j][0] * S.recip[1] + s.bhk[j][1] * S.recip[3];
      arg = S.gamma * S.gamma - (qx * qx + qy * qy);
    }
    s.g2s[j] = arg;
  }
  __syncthreads();
  typename C::Base base;
  C::template bases<F32>(base, S.hd, S.kd, w, lane);
  // Z0 = [I; i Gamma] (spans the columns of S^{-1}[I; O] of Algorithm 1); in
  // a group launch each workgroup writes its share of the rows
  for (int e = tid + XT * g; e < NXT * NXT; e += XT * G) {
    const int row = e / NXT, col = e - row * NXT;
    const double g2v = s.g2s[row];
    const bool dgn = row == col;
    gst(&cg[e], make_double2(dgn ? 1.0 : 0.0, 0.0));
    gst(&dg[e], make_double2((dgn && g2v < 0.0) ? sqrt(-g2v) : 0.0, (dgn && g2v >= 0.0) ? sqrt(g2v) : 0.0));
  }
  if constexpr (GRP) xl_group_sync<C>(cnt, G * ++nsync, failw);
  else __syncthreads();
  int nrhst = 0;
#pragma unroll 1
  for (int i = 0; i < L; ++i) {
    if constexpr (SAVE) {
      if ((i % a.ck.every) == 0) {
        double2* st = reinterpret_cast<double2*>(pws + (long long)(i / a.ck.every) * a.ck.state_bytes);
        if constexpr (GRP) {
          xl_copy_cols(st, cg, g, G);
          xl_copy_cols(st + NX * NX, dg, g, G);
        } else {
          xl_copy(st, cg);
          xl_copy(st + NX * NX, dg);
        }
      }
    }
    C::template slice<STEPPER>(cg, dg, gm, Us, i * T::nodes, S.box, h, N, base, g, G);
    if constexpr (GRP) {
      // the row-sum partials of every workgroup of the pair, summed in the
      // same order everywhere (two buffers: a workgroup cannot be a slice ahead)
      double* part = reinterpret_cast<double*>(wm + C::WG_PART) + 2 * NXT * (i & 1);
      for (int j = tid; j < NXT; j += XT) {
        part[j] = s.rdg[j];
        part[NXT + j] = s.rof[j];
      }
      xl_group_sync<C>(cnt, G * ++nsync, failw);
      for (int j = tid; j < NXT; j += XT) {
        double dv = 0.0, ov = 0.0;
        for (int q = 0; q < G; ++q) {
          const double* pq = reinterpret_cast<const double*>(X.wg_mem + ((long long)pi * G + q) * C::WG_BYTES +
                                                             C::WG_PART) + 2 * NXT * (i & 1);
          dv += pq[j];
          ov += pq[NXT + j];
        }
        s.rdg[j] = dv;
        s.rof[j] = ov;
      }
      __syncthreads();
    }
    // condition estimate of Q = c (Sec. 3.2): the Gershgorin / Varah bound
    double hi = 0.0, lo = 1.0e308;
#pragma unroll
    for (int q = 0; q < XST; ++q) {
      const int row = 64 * q + lane;
      if (row < N) {
        const double dv = s.rdg[row], ov = s.rof[row];
        hi = fmax(hi, dv + ov);
        lo = fmin(lo, dv - ov);
      }
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      hi = fmax(hi, __shfl_xor(hi, o, 64));
      lo = fmin(lo, __shfl_xor(lo, o, 64));
    }
    const double xi = lo > 0.0 ? hi / lo : INFINITY;
    if constexpr (SAVE) {
      if (tid == 0 && g == 0) pws[a.ck.flags_off + i] = xi > a.threshold ? 1 : 0;
    }
    if (xi > a.threshold) {
      ++nrhst;
      if constexpr (GRP) {
        // the elimination spread over the group (ends after a barrier); all
        // then replay it on their row blocks of P
        xl_group_elim<C>(cg, dg, frec, pivg, N, g, G, cnt, nsync, eblk);
        {
          for (int j = tid; j < NXT; j += XT) {
            // brought into range: after a failed barrier the list may be stale
            s.pcrec[j] = (int)((unsigned)pivg[j] % (unsigned)NXT);
            s.pos[j] = j;
          }
          __syncthreads();
          for (int j = tid; j < N; j += XT) s.pos[s.pcrec[j]] = j;
          __syncthreads();
        }
        xl_replay_p<C>(cg, dg, frec, N, g, G);
        if constexpr (SAVE) {
          // T: row block b of I by workgroup (nbp + b) mod G; R: row block b
          // of P Q^{-1} (the replay's blocks) by workgroup b mod G, the one
          // that replayed it
          const int nbp = (N + XW * XCfg::XEMT - 1) / (XW * XCfg::XEMT);
          xl_replay_identity(reinterpret_cast<double2*>(pws + a.ck.q_off + (long long)i * MATB), frec, N,
                             ((g - nbp) % G + G) % G, G);
          if (a.ck.r_off)
            xl_copy_rows<XW * C::XEMT>(reinterpret_cast<double2*>(pws + a.ck.r_off + (long long)i * MATB), dg, g, G);
        }
        xl_group_sync<C>(cnt, G * ++nsync, failw);
      } else {
        xl_elim_record<typename C::ElimCfg>(cg, dg, frec, N, 0);
        if constexpr (SAVE)
          xl_replay_identity(reinterpret_cast<double2*>(pws + a.ck.q_off + (long long)i * MATB), frec, N, 0, 1);
        xl_replay_p<C>(cg, dg, frec, N, 0, 1);
        if constexpr (SAVE) {
          if (a.ck.r_off) {  // R = P Q^{-1} for an adjoint that keeps states only every few slices
            xl_copy(reinterpret_cast<double2*>(pws + a.ck.r_off + (long long)i * MATB), dg);
            __syncthreads();
          }
        }
      }
    }
  }
  if constexpr (SAVE) {  // the final state (the reflection below only reads c and c')
    double2* st = reinterpret_cast<double2*>(pws + (long long)(a.ck.max_ckpt - 1) * a.ck.state_bytes);
    if constexpr (GRP) {
      xl_copy_cols(st, cg, g, G);
      xl_copy_cols(st + NX * NX, dg, g, G);
    } else {
      xl_copy(st, cg);
      xl_copy(st + NX * NX, dg);
    }
  }
  if constexpr (GRP) {
    if (g != 0) return;  // workgroup 0 solves the reflection
  }
  // reflection (Eq. vrhocomp): upper = Gamma Q - iP, lower = Gamma Q + iP,
  // rho = lower x with upper x = e_1
  xl_elim_record<typename C::ElimCfg>(cg, dg, frec, N, 1);
  if constexpr (SAVE) xl_replay_identity(reinterpret_cast<double2*>(pws + a.ck.binv_off), frec, N, 0, 1);
  if (w == 0) {
    // x = E e_{pc_0}: the recorded operations in reverse order, each v <- v - e_pc (f . v)
    const int pc0 = s.pcrec[0];
    double2 v[XST];
#pragma unroll
    for (int q = 0; q < XST; ++q) v[q] = make_double2(64 * q + lane == pc0 ? 1.0 : 0.0, 0.0);
#pragma unroll 1
    for (int k = N - 1; k >= 0; --k) {
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int q = 0; q < XST; ++q) {
        const double2 f = gld(&frec[k * NXT + 64 * q + lane]);
        sr += f.x * v[q].x - f.y * v[q].y;
        si += f.x * v[q].y + f.y * v[q].x;
      }
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        sr += __shfl_xor(sr, o, 64);
        si += __shfl_xor(si, o, 64);
      }
      const int pc = __builtin_amdgcn_readfirstlane(s.pcrec[k]);
      if (lane == (pc & 63)) {
#pragma unroll
        for (int q = 0; q < XST; ++q)
          if (q == (pc >> 6)) v[q] = make_double2(v[q].x - sr, v[q].y - si);
      }
    }
#pragma unroll
    for (int q = 0; q < XST; ++q) s.xv[64 * q + lane] = v[q];
  }
  if (tid == 0) {
    s.bnorm_bits = 0;
    s.xnorm_bits = 0;
  }
  __syncthreads();
  // row j of the reflection's outputs (a thread per row, or a loop over rows
  // when the width exceeds the workgroup)
  auto out_row = [&](int j) {
    double eta = 0.0;
    double2 rj = make_double2(0.0, 0.0);
    if (j < N) {
      const double g2v = s.g2s[j];
      const double g_r = g2v >= 0.0 ? sqrt(g2v) : 0.0, g_i = g2v >= 0.0 ? 0.0 : -sqrt(-g2v);
      double rs = 0.0;  // row j of Gamma Q - iP, for the breakdown test
      for (int k = 0; k < N; ++k) {
        const double2 cv = gld(&cg[j * NXT + k]), pv = gld(&dg[j * NXT + k]), x = s.xv[k];
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
      if (rs == rs) atomicMax(&s.bnorm_bits, (unsigned long long)__double_as_longlong(rs));
      if (xm == xm) atomicMax(&s.xnorm_bits, (unsigned long long)__double_as_longlong(xm));
    }
    a.intensity[(long long)p * a.ld + j] = eta;
    if (a.rho) a.rho[(long long)p * a.ld + j] = rj;
  };
  if constexpr (NXT <= XT) {
    if (tid < a.ld) out_row(tid);
  } else {
    for (int j = tid; j < a.ld; j += XT) out_row(j);
  }
  __syncthreads();
  const bool brk = !(__longlong_as_double((long long)s.bnorm_bits) * __longlong_as_double((long long)s.xnorm_bits) <=
                     BREAKDOWN_COND);
  bool lost = false;
  if constexpr (GRP)
    lost = s.sync_fail || __hip_atomic_load(failw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
  const int stv = lost ? 3 : s.flag_singular ? 1 : s.bad ? 2 : brk ? 4 : 0;
  if (stv != 0) {  // a failed pair's outputs are NaN
    for (int j = tid; j < N; j += XT) {
      a.intensity[(long long)p * a.ld + j] = NAN;
      if (a.rho) a.rho[(long long)p * a.ld + j] = make_double2(NAN, NAN);
    }
  }
  if (tid == 0) {
    a.status[p] = stv;
    if (a.nrhst) a.nrhst[p] = nrhst;
  }
}

template <int STEPPER, bool SAVE>
__global__ __launch_bounds__(XT, 1) void forward_xl_kernel(LargeArgs A) {
  char* slot = A.scratch + (long long)blockIdx.x * XSLOT_BYTES;
#pragma unroll 1
  for (int pi = blockIdx.x; pi < A.f.n_pairs; pi += gridDim.x) {
    const int p = A.f.pair_list ? A.f.pair_list[pi] : pi;
    xl_run_pair<XCfg, STEPPER, false, SAVE>(A, p, slot, XlGroup{}, 0, 0);
    __syncthreads();  // LDS is reused by the next pair
  }
}

// Group launch: G workgroups per pair, grid = pairs x G, all resident
// (cooperative launch).
template <int STEPPER, bool SAVE>
__global__ __launch_bounds__(XT, 1) void forward_xl_group_kernel(LargeArgs A, XlGroup X) {
  const int pi = blockIdx.x / X.group, g = blockIdx.x - pi * X.group;
  const int p = A.f.pair_list ? A.f.pair_list[pi] : pi;
  xl_run_pair<XCfg, STEPPER, true, SAVE>(A, p, nullptr, X, pi, g);
}

__global__ void xl_group_reset_kernel(unsigned* counters, int n) {
  for (int e = threadIdx.x; e < XG_CTR_WORDS * n; e += blockDim.x) counters[e] = 0u;
}

}  // namespace

hipError_t launch_forward_xl(int stepper, const LargeArgs& a, hipStream_t stream) {
  if (a.f.n_pairs < 1) return hipSuccess;
  const int grid = a.f.n_pairs < a.n_slots ? a.f.n_pairs : a.n_slots;
  if (grid < 1 || (stepper != 0 && stepper != 1 && stepper != (0 | F32_STAGES) && stepper != (1 | F32_STAGES)))
    return hipErrorInvalidValue;
  const bool save = a.f.ws != nullptr;
  if (save && (stepper & F32_STAGES)) return hipErrorInvalidValue;
  if (stepper == 0 && save)
    hipLaunchKernelGGL((forward_xl_kernel<0, true>), dim3(grid), dim3(XT), 0, stream, a);
  else if (stepper == 0)
    hipLaunchKernelGGL((forward_xl_kernel<0, false>), dim3(grid), dim3(XT), 0, stream, a);
  else if (stepper == 1 && save)
    hipLaunchKernelGGL((forward_xl_kernel<1, true>), dim3(grid), dim3(XT), 0, stream, a);
  else if (stepper == 1)
    hipLaunchKernelGGL((forward_xl_kernel<1, false>), dim3(grid), dim3(XT), 0, stream, a);
  else if (stepper == (0 | F32_STAGES))
    hipLaunchKernelGGL((forward_xl_kernel<0 | F32_STAGES, false>), dim3(grid), dim3(XT), 0, stream, a);
  else
    hipLaunchKernelGGL((forward_xl_kernel<1 | F32_STAGES, false>), dim3(grid), dim3(XT), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_forward_xl_group(int stepper, const LargeArgs& a, const XlGroup& x, hipStream_t stream) {
  if (a.f.n_pairs < 1) return hipSuccess;
  const bool save = a.f.ws != nullptr;
  const void* f = nullptr;
  if (stepper == 0) f = save ? reinterpret_cast<const void*>(&forward_xl_group_kernel<0, true>)
                             : reinterpret_cast<const void*>(&forward_xl_group_kernel<0, false>);
  else if (stepper == 1) f = save ? reinterpret_cast<const void*>(&forward_xl_group_kernel<1, true>)
                                  : reinterpret_cast<const void*>(&forward_xl_group_kernel<1, false>);
  else if (stepper == (0 | F32_STAGES) && !save)
    f = reinterpret_cast<const void*>(&forward_xl_group_kernel<0 | F32_STAGES, false>);
  else if (stepper == (1 | F32_STAGES) && !save)
    f = reinterpret_cast<const void*>(&forward_xl_group_kernel<1 | F32_STAGES, false>);
  if (x.group < 1 || !f) return hipErrorInvalidValue;
  hipLaunchKernelGGL(xl_group_reset_kernel, dim3(1), dim3(256), 0, stream, x.counters, a.f.n_pairs);
  LargeArgs aa = a;
  XlGroup xx = x;
  void* params[] = {&aa, &xx};
  return hipLaunchCooperativeKernel(f, dim3(a.f.n_pairs * x.group), dim3(XT), params, 0, stream);
}

int forward_xl_group_max_workgroups(int device) {
  int coop = 0, cus = 0, p[4] = {0, 0, 0, 0};
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) != hipSuccess || !coop) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&p[0], forward_xl_group_kernel<0, false>, XT, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&p[1], forward_xl_group_kernel<1, false>, XT, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&p[2], forward_xl_group_kernel<0, true>, XT, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&p[3], forward_xl_group_kernel<1, true>, XT, 0) != hipSuccess)
    return 0;
  int per = p[0];
  for (int q = 1; q < 4; ++q) per = p[q] < per ? p[q] : per;
  return cus * (per > 0 ? per : 0);
}

int forward_xl_slots(int device) {
  int cus = 0, p0 = 0, p1 = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  int p2 = 0, p3 = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&p0, forward_xl_kernel<0, false>, XT, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&p1, forward_xl_kernel<1, false>, XT, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&p2, forward_xl_kernel<0, true>, XT, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&p3, forward_xl_kernel<1, true>, XT, 0) != hipSuccess)
    return 0;
  p0 = p0 < p2 ? p0 : p2;
  p1 = p1 < p3 ? p1 : p3;
  const int per = p0 < p1 ? p0 : p1;
  return cus * (per > 0 ? per : 0);
}

}  // namespace rheed
