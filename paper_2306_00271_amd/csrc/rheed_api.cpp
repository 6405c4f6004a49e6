// Host side of the C ABI declared in include/rheed.h: argument validation,
// plan construction (descriptor upload) and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "rheed.h"
#include "rheed_internal.h"
#include "rheed_large.h"


using namespace rheed;

static_assert(RHEED_NOALLOC_MAX_ATOMS == PBWD_STATIC_ATOMS, "header and fixed array disagree");

namespace {
thread_local std::string g_last_error;

rheed_status fail(rheed_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}
rheed_status hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return RHEED_E_HIP;
}

// CODATA 2018
constexpr double kMe = 9.1093837015e-31, kQe = 1.602176634e-19, kHbar = 1.054571817e-34, kC = 299792458.0;
}  // namespace

struct rheed_plan_s {
  rheed_opts opts{};
  int n_struct = 0, n_pairs = 0, max_beams = 0, nodes_per_slice = 0;
  double cset[12] = {};
  double sp_a[3] = {0, 0, 0}, sp_b[4] = {0, 0, 0, 0};  // SP4 weights of the N > 64 kernel
  bool splitting = false;    // a splitting stepper (Sec. 3.4)
  SplitSteps sp{};           // its steps on the one-workgroup kernel (N <= 64)
  long long table_elems = 0, n_atoms_total = 0, max_table = 0;
  std::vector<StructDev> hs;
  std::vector<int> beams, pair_struct;
  std::vector<long long> table_off, atom_off, atom_struct;
  std::vector<int> bin_ptr, bin_jk;
  CkptLayout ck{};   // states kept for the adjoint, pairs with N <= 64 (matrices padded to 64)
  CkptLayout ckl{};  // the same for pairs with 64 < N <= 128 (padded to 128); same pair stride
  CkptLayout ckx{};  // and for pairs with 128 < N <= 256 (padded to 256)
  size_t fwd_ws = 0, bwd_ws = 0;
  StructDev* d_structs = nullptr;
  int* d_beams = nullptr;
  int* d_pair_struct = nullptr;
  long long* d_atom_struct = nullptr;
  int* d_bin_ptr = nullptr;
  int* d_bin_jk = nullptr;
  double* d_pbwd = nullptr;  // partial sums of the potential adjoint
  char* d_xch = nullptr;     // exchange blocks of the split layout
  int xch_give_up = -1;      // rheed_plan_force_sync_failure: the half whose first wait fails at once
  bool split = false;
  int split_max = 0;
  long long g_pair_stride = 0;  // adjoint stage buffer elements per pair
  int max_nodes = 0;
  size_t xs_off = 0;            // adjoint workspace: x of a segment's transformed states
  // pairs of structures with N <= 64 (propagated by the one- and two-workgroup
  // kernels) and with 64 < N <= 128 (the large kernel), in pair order
  std::vector<int> small_pairs, large_pairs;
  // pairs of structures with 128 < N <= 256 (forward only, their own kernel)
  std::vector<int> xl_pairs;
  int* d_xl_pairs = nullptr;
  char* d_xscratch = nullptr;    // per resident workgroup of that kernel: its state slot
  int xl_slots = 0;
  // small batches: a group of xl_group workgroups per pair (1: one workgroup per pair)
  int xl_group = 1;
  char* d_xg_pair = nullptr;
  char* d_xg_wg = nullptr;
  unsigned* d_xg_cnt = nullptr;
  // pairs of structures with 256 < N <= 576 (forward only): a group launch of
  // xxl_group workgroups per pair
  std::vector<int> xxl_pairs;
  int* d_xxl_pairs = nullptr;
  int xxl_group = 1;
  int xxl_per_launch = 0;        // pairs per launch (all resident at once); larger batches take several
  char* d_xxg_pair = nullptr;
  char* d_xxg_wg = nullptr;
  unsigned* d_xxg_cnt = nullptr;
  int* d_small_pairs = nullptr;  // only when both kinds are present
  int* d_large_pairs = nullptr;  // in cost order (dearest first)
  int* d_large_plain = nullptr;  // in pair order
  bool large_cost_order = true;  // which of the two lists rheed_forward uses
  char* d_lscratch = nullptr;    // per resident workgroup of the large kernel: its state slot
  int large_slots = 0;
  int scratch_slots = 0;         // slots allocated: max of large_slots and queue_grid
  // one persistent launch over a batch mixing N <= 64 and N > 64 (RK, FP64)
  bool queue_ok = false;         // the batch can run on forward_queue_kernel
  bool use_queue = false;        // rheed_forward runs it (autotune may switch it off)
  int queue_grid = 0;            // its workgroups
  int* d_queue_order = nullptr;  // every pair, dearest first
  int* d_queue_counter = nullptr;
  std::vector<int> large_plain;
  std::vector<int> queue_order;
};

namespace {

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// extra workspace of rheed_bulk_reflection beyond fwd_ws: intensities and
// status of each layer's forward pass, the done flags
size_t bulk_extra(const rheed_plan_s* P) {
  const size_t np = (size_t)P->n_pairs, m = (size_t)P->max_beams;
  return align256(np * m * 8) + 2 * align256(np * 4);
}

}  // namespace

extern "C" {

const char* rheed_status_string(rheed_status s) {
  switch (s) {
    case RHEED_OK: return "ok";
    case RHEED_E_INVALID: return "invalid argument";
    case RHEED_E_HIP: return "HIP runtime error";
    case RHEED_E_NOMEM: return "out of memory";
    case RHEED_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* rheed_last_error(void) { return g_last_error.c_str(); }

rheed_status rheed_beam_constants(double energy_eV, double* gamma, double* kappa) {
  if (!(energy_eV > 0.0) || !gamma || !kappa) return fail(RHEED_E_INVALID, "energy must be > 0 and outputs non-null");
  const double e = kQe * energy_eV;
  const double p2 = 2.0 * kMe * e * (1.0 + e / (2.0 * kMe * kC * kC));
  *gamma = std::sqrt(p2) / kHbar * 1e-10;
  *kappa = 2.0 * kMe * kQe / (kHbar * kHbar) * (1.0 + e / (kMe * kC * kC)) * 1e-20;
  return RHEED_OK;
}

rheed_status rheed_plan_create(rheed_plan_t* out, const rheed_opts* opts, int32_t n_struct,
                               const rheed_structure* structs, const int32_t* angles_per_struct) {
  if (!out || !opts || !structs || !angles_per_struct || n_struct < 1)
    return fail(RHEED_E_INVALID, "plan_create: null argument or n_struct < 1");
  *out = nullptr;
  if (opts->stepper < RHEED_RK4 || opts->stepper > RHEED_SP6_ABA) return fail(RHEED_E_INVALID, "unknown stepper");
  const bool splitting = opts->stepper >= RHEED_SP4;
  if (splitting && opts->layout == RHEED_LAYOUT_SPLIT)
    return fail(RHEED_E_UNSUPPORTED, "the splitting steppers run on the one-workgroup-per-pair kernels only");
  if (!(opts->rhst_threshold >= 1.0)) return fail(RHEED_E_INVALID, "rhst_threshold must be >= 1");
  if (opts->checkpoint_every < 1) return fail(RHEED_E_INVALID, "checkpoint_every must be >= 1");
  if (opts->convention != RHEED_INTENSITY_FLUX && opts->convention != RHEED_INTENSITY_PAPER)
    return fail(RHEED_E_INVALID, "unknown intensity convention");
  if (opts->layout != RHEED_LAYOUT_AUTO && opts->layout != RHEED_LAYOUT_WHOLE && opts->layout != RHEED_LAYOUT_SPLIT)
    return fail(RHEED_E_INVALID, "unknown layout");
  if (opts->stage_precision != RHEED_STAGES_FP64 && opts->stage_precision != RHEED_STAGES_FP32)
    return fail(RHEED_E_INVALID, "unknown stage precision");
  if (opts->stage_precision == RHEED_STAGES_FP32 && splitting)
    return fail(RHEED_E_UNSUPPORTED, "FP32 stage products need an RK stepper");
  auto* P = new rheed_plan_s();
  P->opts = *opts;
  P->n_struct = n_struct;
  if (opts->stepper == RHEED_RK4) {
    P->nodes_per_slice = 2;
    P->cset[0] = 0.0;
    P->cset[1] = 0.5;
  } else if (opts->stepper == RHEED_RK6) {
    P->nodes_per_slice = 4;
    P->cset[0] = 0.0;
    P->cset[1] = 1.0 / 3.0;
    P->cset[2] = 0.5;
    P->cset[3] = 2.0 / 3.0;
  } else {
    // Splitting methods: compositions of Stormer-Verlet steps of lengths
    // alpha_k (sum 1).  Fourth order: the triple jump g1, g2, g1 with
    // 2 g1 + g2 = 1, 2 g1^3 + g2^3 = 0; sixth order: the triple jump of
    // that step, w1, w0, w1 with 2 w1 + w0 = 1, 2 w1^5 + w0^5 = 0, so nine
    // steps w_i g_j.  BAB: drifts alpha_k, kicks their half sums (first and
    // last alpha / 2); ABA: kicks alpha_k, drifts the half sums.
    const double g1 = 1.0 / (2.0 - std::pow(2.0, 1.0 / 3.0)), g2 = 1.0 - 2.0 * g1;
    std::vector<double> steps = {g1, g2, g1};
    if (opts->stepper == RHEED_SP6 || opts->stepper == RHEED_SP6_ABA) {
      const double w1 = 1.0 / (2.0 - std::pow(2.0, 1.0 / 5.0)), w0 = 1.0 - 2.0 * w1;
      std::vector<double> s6;
      for (double w : {w1, w0, w1})
        for (double g : {g1, g2, g1}) s6.push_back(w * g);
      steps = s6;
    }
    std::vector<double> half;
    half.push_back(steps.front() / 2);
    for (size_t k = 0; k + 1 < steps.size(); ++k) half.push_back((steps[k] + steps[k + 1]) / 2);
    half.push_back(steps.back() / 2);
    const bool aba = opts->stepper == RHEED_SP4_ABA || opts->stepper == RHEED_SP6_ABA;
    const std::vector<double>& da = aba ? half : steps;   // drift weights
    const std::vector<double>& kb = aba ? steps : half;   // kick weights
    SplitSteps& sp = P->sp;
    sp.form = aba ? 1 : 0;
    sp.kicks = (int)kb.size();
    for (size_t k = 0; k < da.size(); ++k) sp.a[k] = da[k];
    for (size_t k = 0; k < kb.size(); ++k) sp.b[k] = kb[k];
    // kick positions (in units of h from the slice start) in the order the
    // kicks use them; the distinct ones other than the slice end are the
    // slice's nodes, the slice end is the next slice's first node
    std::vector<double> pos;
    if (aba) {
      double t = 0.0;
      for (int r = 0; r < sp.kicks; ++r) pos.push_back(t += da[r]);
    } else {
      double t = 0.0;
      pos.push_back(0.0);
      for (size_t r = 0; r < da.size(); ++r) pos.push_back(t += da[r]);
    }
    int nps = 0;
    for (int r = 0; r < sp.kicks; ++r) {
      if (!aba && std::fabs(pos[r] - 1.0) < 1e-14) {
        sp.node[r] = -1;  // the slice end
        continue;
      }
      int m = 0;
      while (m < nps && !(std::fabs(pos[r] - P->cset[m]) < 1e-14)) ++m;
      if (m == nps) P->cset[nps++] = pos[r];
      sp.node[r] = m;
    }
    for (int r = 0; r < sp.kicks; ++r)
      if (sp.node[r] < 0) sp.node[r] = nps;
    sp.nps = nps;
    P->nodes_per_slice = nps;
    P->splitting = true;
    // the kernel for N > 64 runs the fourth-order BAB method with these weights
    for (int q = 0; q < 3; ++q) P->sp_a[q] = steps.size() == 3 ? steps[q] : 0.0;
    for (int q = 0; q < 4; ++q) P->sp_b[q] = half.size() == 4 ? half[q] : 0.0;
  }
  int max_l = 0;
  for (int s = 0; s < n_struct; ++s) {
    const rheed_structure& st = structs[s];
    char buf[256];
    if (st.n_beams < 1 || st.n_beams > RHEED_MAX_BEAMS || !st.beam_hk) {
      snprintf(buf, sizeof buf, "structure %d: n_beams must be in [1, %d]", s, RHEED_MAX_BEAMS);
      delete P;
      return fail(RHEED_E_UNSUPPORTED, buf);
    }
    if (opts->stage_precision == RHEED_STAGES_FP32 && st.n_beams > NX) {
      delete P;
      return fail(RHEED_E_UNSUPPORTED, "structure " + std::to_string(s) + ": FP32 stage products need N <= 256");
    }
    if (st.n_beams > NL && splitting) {
      delete P;
      return fail(RHEED_E_UNSUPPORTED, "structure " + std::to_string(s) + ": N > 128 needs an RK stepper");
    }
    if (splitting && st.n_beams > NP && opts->stepper != RHEED_SP4) {
      delete P;
      return fail(RHEED_E_UNSUPPORTED, "structure " + std::to_string(s) +
                                           ": for N > 64 the only splitting stepper is RHEED_SP4");
    }
    if (st.beam_hk[0] != 0 || st.beam_hk[1] != 0) {
      delete P;
      return fail(RHEED_E_INVALID, "structure " + std::to_string(s) + ": beam 0 must be (0, 0)");
    }
    if (st.n_slices < 1 || !(st.thickness > 0.0) || !(st.wavenumber > 0.0) || angles_per_struct[s] < 1) {
      delete P;
      return fail(RHEED_E_INVALID, "structure " + std::to_string(s) + ": need n_slices >= 1, thickness > 0, "
                                   "wavenumber > 0 and at least one angle");
    }
    std::set<std::pair<int, int>> seen;
    int hmin = st.beam_hk[0], hmax = hmin, kmin = st.beam_hk[1], kmax = kmin;
    for (int j = 0; j < st.n_beams; ++j) {
      const int h = st.beam_hk[2 * j], k = st.beam_hk[2 * j + 1];
      if (!seen.insert({h, k}).second) {
        delete P;
        return fail(RHEED_E_INVALID, "structure " + std::to_string(s) + ": duplicate beam");
      }
      hmin = std::min(hmin, h);
      hmax = std::max(hmax, h);
      kmin = std::min(kmin, k);
      kmax = std::max(kmax, k);
    }
    StructDev d{};
    d.n_beams = st.n_beams;
    d.n_slices = st.n_slices;
    d.hd = hmax - hmin;
    d.kd = kmax - kmin;
    d.box = (2 * d.hd + 1) * (2 * d.kd + 1);
    const int box_max = (st.n_beams <= NP) ? MAXBOX : (st.n_beams <= NL) ? MAXBOXL : (st.n_beams <= NX) ? MAXBOXX
                                                                                                     : MAXBOXXX;
    if (d.box > box_max) {
      delete P;
      return fail(RHEED_E_UNSUPPORTED, "structure " + std::to_string(s) + ": rod-difference table row of " +
                                           std::to_string(d.box) + " entries exceeds " + std::to_string(box_max) +
                                           " for N = " + std::to_string(st.n_beams));
    }
    d.n_nodes = st.n_slices * P->nodes_per_slice + 1;
    // (j, k) pairs of every rod difference g_j - g_k, grouped by table entry,
    // for the adjoint's gradient assembly: j * Wp + k, Wp the padded beam
    // count of the structure's kernels (64 or 128)
    {
      const int W = 2 * d.kd + 1;
      const int Wp = st.n_beams <= NP ? NP : st.n_beams <= NL ? NL : st.n_beams <= NX ? NX : NXX;
      std::vector<std::vector<int>> lists(d.box);
      for (int j = 0; j < st.n_beams; ++j)
        for (int k = 0; k < st.n_beams; ++k) {
          const int dh = st.beam_hk[2 * j] - st.beam_hk[2 * k], dk = st.beam_hk[2 * j + 1] - st.beam_hk[2 * k + 1];
          lists[(dh + d.hd) * W + (dk + d.kd)].push_back(j * Wp + k);
        }
      d.bin_ptr_off = (int)P->bin_ptr.size();
      d.bin_jk_off = (int)P->bin_jk.size();
      int acc = 0;
      for (int b = 0; b < d.box; ++b) {
        P->bin_ptr.push_back(acc);
        for (int v : lists[b]) P->bin_jk.push_back(v);
        acc += (int)lists[b].size();
      }
      P->bin_ptr.push_back(acc);
    }
    d.n_atoms = std::max(0, st.n_atoms);
    d.beam_off = (int)(P->beams.size() / 2);
    for (int j = 0; j < 2 * st.n_beams; ++j) P->beams.push_back(st.beam_hk[j]);
    d.pair_off = P->n_pairs;
    d.n_angles = angles_per_struct[s];
    d.h = st.thickness / st.n_slices;
    d.thickness = st.thickness;
    d.gamma = st.wavenumber;
    for (int c = 0; c < 4; ++c) d.recip[c] = st.recip[c];
    d.table_off = P->table_elems;
    d.atom_off = P->n_atoms_total;
    for (int m = 0; m < 4; ++m) {
      d.scat_a[m] = st.scat_a[m];
      d.scat_b[m] = st.scat_b[m];
    }
    // slab-mean rescaling s (position independent) and u = kappa s (charge - i alpha) V_g
    if (d.n_atoms > 0) {
      double per_atom = 0.0;
      for (int m = 0; m < 4; ++m) {
        if (!(st.scat_b[m] > 0.0)) {
          delete P;
          return fail(RHEED_E_INVALID, "structure " + std::to_string(s) + ": scat_b must be > 0");
        }
        per_atom += st.scat_a[m] * std::pow(M_PI / st.scat_b[m], 1.5);
      }
      if (!(st.cell_area > 0.0) || per_atom == 0.0) {
        delete P;
        return fail(RHEED_E_INVALID, "structure " + std::to_string(s) + ": bad potential model");
      }
      const double raw = d.n_atoms * per_atom / (st.cell_area * st.thickness);
      const double sc = st.mean_inner_potential / raw;
      d.pref_re = st.kappa * sc * st.charge / st.cell_area;
      d.pref_im = -st.kappa * sc * st.absorption / st.cell_area;
    }
    P->hs.push_back(d);
    P->table_off.push_back(P->table_elems);
    P->atom_off.push_back(P->n_atoms_total);
    for (int a = 0; a < d.n_atoms; ++a) P->atom_struct.push_back(s);
    P->table_elems += (long long)d.n_nodes * d.box;
    P->max_table = std::max(P->max_table, (long long)d.n_nodes * d.box);
    P->max_nodes = std::max(P->max_nodes, d.n_nodes);
    P->n_atoms_total += d.n_atoms;
    for (int a = 0; a < angles_per_struct[s]; ++a) {
      ((st.n_beams <= NP) ? P->small_pairs : (st.n_beams <= NL) ? P->large_pairs
                                           : (st.n_beams <= NX) ? P->xl_pairs : P->xxl_pairs)
          .push_back(P->n_pairs + a);
      P->pair_struct.push_back(s);
    }
    P->n_pairs += angles_per_struct[s];
    P->max_beams = std::max(P->max_beams, st.n_beams);
    max_l = std::max(max_l, st.n_slices);
  }
  P->table_off.push_back(P->table_elems);
  P->atom_off.push_back(P->n_atoms_total);
  // per-pair checkpoint block: the state at the start of every segment and
  // the final state, T = Q^{-1} of every transformation, with segments
  // longer than one slice also R = P Q^{-1} (the normalised P) of every
  // transformation, and one decision byte per slice
  // (with N > 64 also B^{-1} of the reflection solve); the layout of the
  // pairs with N > 64 pads every matrix to 128, and both kinds share the
  // larger pair stride
  auto layout = [&](int w, bool binv) {
    CkptLayout c{};
    c.every = opts->checkpoint_every;
    c.max_ckpt = (max_l + opts->checkpoint_every - 1) / opts->checkpoint_every + 1;
    c.state_bytes = (long long)2 * w * w * sizeof(double2);
    const long long mat = (long long)w * w * sizeof(double2), slot_bytes = (long long)max_l * mat;
    c.q_off = c.max_ckpt * c.state_bytes;
    // a splitting method keeps R at every K: the BAB method's final kick changes
    // the final state, which therefore cannot stand for the last slice's R
    const bool rslots = c.every > 1 || P->splitting;
    c.r_off = rslots ? c.q_off + slot_bytes : 0;
    const long long end = (rslots ? c.r_off : c.q_off) + slot_bytes;
    c.binv_off = binv ? end : 0;
    c.flags_off = end + (binv ? mat : 0);
    c.pair_stride = ((c.flags_off + max_l + 255) / 256) * 256;
    return c;
  };
  const bool wide = !P->large_pairs.empty(), xwide = !P->xl_pairs.empty();
  P->ck = layout(NP, false);
  long long stride = P->ck.pair_stride;
  if (wide) {
    P->ckl = layout(NL, true);
    stride = std::max(stride, P->ckl.pair_stride);
  }
  if (xwide) {
    P->ckx = layout(NX, true);
    stride = std::max(stride, P->ckx.pair_stride);
  }
  P->ck.pair_stride = P->ckl.pair_stride = P->ckx.pair_stride = stride;
  const int wmax = xwide ? NX : wide ? NL : NP;
  P->fwd_ws = (size_t)P->ck.pair_stride * P->n_pairs;
  // adjoint stage buffer: (v_r, g_r) of every stage of every slice; for a
  // splitting method of every kick it keeps per slice (the BAB method's final
  // kick in one more slice)
  if (P->splitting) {
    const int nks = P->sp.form == 0 ? P->sp.kicks - 1 : P->sp.kicks;
    P->g_pair_stride = (long long)(max_l + 1) * nks * 2 * wmax;
  } else {
    P->g_pair_stride = (long long)max_l * (P->opts.stepper == RHEED_RK4 ? 4 : 7) * 2 * wmax;
  }
  P->bwd_ws = (size_t)P->g_pair_stride * sizeof(double2) * P->n_pairs;
  if (P->ck.every > 1) {  // x at the transformed states of a segment
    P->xs_off = P->bwd_ws;
    P->bwd_ws += (size_t)P->ck.every * wmax * sizeof(double2) * P->n_pairs;
  }

  // the N > 64 kernel takes its pairs dearest first: cost ~ (column blocks)^2 x slices
  P->large_plain = P->large_pairs;
  if (!P->large_pairs.empty()) {
    auto cost = [&](int p) {
      const StructDev& d = P->hs[P->pair_struct[p]];
      const long long nb = (d.n_beams + 15) / 16;
      return nb * nb * d.n_slices;
    };
    std::stable_sort(P->large_pairs.begin(), P->large_pairs.end(), [&](int x, int y) { return cost(x) > cost(y); });
  }
  // the queue of the one-launch path: every pair by estimated cost, dearest
  // first (per slice about 9.5 us x (column blocks)^2 on the large path and
  // 60 us on the one-workgroup path, as measured on MI355X)
  {
    auto qcost = [&](int p) {
      const StructDev& d = P->hs[P->pair_struct[p]];
      const double nb = (d.n_beams + 15) / 16;
      return d.n_slices * (d.n_beams > NP ? 9.5 * nb * nb : 60.0);
    };
    P->queue_order.resize(P->n_pairs);
    for (int p = 0; p < P->n_pairs; ++p) P->queue_order[p] = p;
    std::stable_sort(P->queue_order.begin(), P->queue_order.end(), [&](int x, int y) { return qcost(x) > qcost(y); });
  }
  // the adjoint and its state saving: FP64, the RK steppers for every N and
  // the splitting methods for N <= 64
  if ((P->splitting && !P->large_pairs.empty()) || opts->stage_precision != RHEED_STAGES_FP64 ||
      !P->xxl_pairs.empty()) {
    P->fwd_ws = 0;
    P->bwd_ws = 0;
  }

  // split layout: two workgroups per pair, both resident (cooperative launch)
  const int n_small = (int)P->small_pairs.size(), n_large = (int)P->large_pairs.size();
  {
    int dev = 0;
    const bool have_dev = hipGetDevice(&dev) == hipSuccess;
    P->split_max = have_dev ? forward_split_max_pairs(dev) : 0;
    P->split = opts->layout != RHEED_LAYOUT_WHOLE && !P->splitting && n_small > 0 && n_small <= P->split_max;
    if (n_large > 0) {
      const int slots = have_dev ? forward_large_slots(dev) : 0;
      if (slots < 1) {
        delete P;
        return fail(RHEED_E_HIP, "the kernel for N > 64 cannot be resident on this device");
      }
      P->large_slots = std::min(n_large, slots);
      P->scratch_slots = P->large_slots;
      P->queue_ok = n_small > 0 && !P->splitting && opts->stage_precision == RHEED_STAGES_FP64 &&
                    opts->layout != RHEED_LAYOUT_SPLIT && P->xl_pairs.empty() && P->xxl_pairs.empty();
      if (P->queue_ok) {
        const int qs = forward_queue_slots(dev);
        P->queue_ok = qs > 0;
        P->queue_grid = std::min(P->n_pairs, qs);
        P->scratch_slots = std::max(P->scratch_slots, P->queue_grid);
        P->use_queue = P->queue_ok;
      }
    }
    if (!P->xl_pairs.empty()) {
      const int slots = have_dev ? forward_xl_slots(dev) : 0;
      if (slots < 1) {
        delete P;
        return fail(RHEED_E_HIP, "the kernel for N > 128 cannot be resident on this device");
      }
      P->xl_slots = std::min((int)P->xl_pairs.size(), slots);
      // a batch that cannot fill the device runs each pair on a group of
      // workgroups (one per 16-column block at most), as many as fit at once
      int maxn = 0;
      for (int q : P->xl_pairs) maxn = std::max(maxn, P->hs[P->pair_struct[q]].n_beams);
      const int n_xl = (int)P->xl_pairs.size();
      const int cap = opts->layout != RHEED_LAYOUT_WHOLE ? forward_xl_group_max_workgroups(dev) : 0;
      const int g = std::min((maxn + 15) / 16, cap / n_xl);
      P->xl_group = g >= 2 ? g : 1;
    }
    if (!P->xxl_pairs.empty()) {
      // every pair on a cooperative group, as many pairs per launch as the
      // device holds at once (a larger batch takes several launches, which
      // reuse the group memory)
      const int cap = have_dev ? forward_xxl_group_max_workgroups(dev) : 0;
      if (cap < 1) {
        delete P;
        return fail(RHEED_E_HIP, "the kernel for N > 256 cannot be resident on this device");
      }
      const int n_xxl = (int)P->xxl_pairs.size();
      int maxn = 0;
      for (int q : P->xxl_pairs) maxn = std::max(maxn, P->hs[P->pair_struct[q]].n_beams);
      P->xxl_group = std::max(1, std::min((maxn + 15) / 16, cap / std::min(n_xxl, cap)));
      P->xxl_per_launch = std::min(n_xxl, cap / P->xxl_group);
    }
    if (opts->layout == RHEED_LAYOUT_SPLIT && !P->split && n_small > 0) {
      const int mx = P->split_max;
      delete P;
      return fail(RHEED_E_UNSUPPORTED, "layout SPLIT holds at most " + std::to_string(mx) + " pairs on this device");
    }
  }

  hipError_t e;
  if ((e = hipMalloc(&P->d_structs, sizeof(StructDev) * P->hs.size())) != hipSuccess ||
      (e = hipMalloc(&P->d_beams, sizeof(int) * P->beams.size())) != hipSuccess ||
      (e = hipMalloc(&P->d_pair_struct, sizeof(int) * P->pair_struct.size())) != hipSuccess ||
      (e = hipMalloc(&P->d_atom_struct, sizeof(long long) * std::max<size_t>(1, P->atom_struct.size()))) != hipSuccess ||
      (e = hipMalloc(&P->d_bin_ptr, sizeof(int) * P->bin_ptr.size())) != hipSuccess ||
      (e = hipMalloc(&P->d_bin_jk, sizeof(int) * P->bin_jk.size())) != hipSuccess ||
      (e = hipMalloc(&P->d_pbwd, sizeof(double) * 3 * PBWD_CHUNKS * std::max<long long>(1, P->n_atoms_total))) !=
          hipSuccess ||
      (P->split && (e = hipMalloc(&P->d_xch, (size_t)XCH_STRIDE * n_small)) != hipSuccess) ||
      ((n_large > 0 || !P->xl_pairs.empty()) && n_small > 0 &&
       (e = hipMalloc(&P->d_small_pairs, sizeof(int) * n_small)) != hipSuccess) ||
      (!P->xl_pairs.empty() && (e = hipMalloc(&P->d_xl_pairs, sizeof(int) * P->xl_pairs.size())) != hipSuccess) ||
      (!P->xl_pairs.empty() &&
       (e = hipMalloc(&P->d_xscratch, (size_t)XSLOT_BYTES * P->xl_slots)) != hipSuccess) ||
      (P->xl_group > 1 &&
       (e = hipMalloc(&P->d_xg_pair, (size_t)XG_PAIR_BYTES * P->xl_pairs.size())) != hipSuccess) ||
      (P->xl_group > 1 &&
       (e = hipMalloc(&P->d_xg_wg, (size_t)XG_WG_BYTES * P->xl_group * P->xl_pairs.size())) != hipSuccess) ||
      (P->xl_group > 1 &&
       (e = hipMalloc(&P->d_xg_cnt, sizeof(unsigned) * XG_CTR_WORDS * P->xl_pairs.size())) != hipSuccess) ||
      (!P->xxl_pairs.empty() &&
       (e = hipMalloc(&P->d_xxl_pairs, sizeof(int) * P->xxl_pairs.size())) != hipSuccess) ||
      (!P->xxl_pairs.empty() &&
       (e = hipMalloc(&P->d_xxg_pair, (size_t)XXG_PAIR_BYTES * P->xxl_per_launch)) != hipSuccess) ||
      (!P->xxl_pairs.empty() &&
       (e = hipMalloc(&P->d_xxg_wg, (size_t)XXG_WG_BYTES * P->xxl_group * P->xxl_per_launch)) != hipSuccess) ||
      (!P->xxl_pairs.empty() &&
       (e = hipMalloc(&P->d_xxg_cnt, sizeof(unsigned) * XG_CTR_WORDS * P->xxl_per_launch)) != hipSuccess) ||
      (n_large > 0 && (e = hipMalloc(&P->d_large_pairs, sizeof(int) * n_large)) != hipSuccess) ||
      (n_large > 0 && (e = hipMalloc(&P->d_large_plain, sizeof(int) * n_large)) != hipSuccess) ||
      (n_large > 0 && (e = hipMalloc(&P->d_lscratch, (size_t)LSLOT_BYTES * P->scratch_slots)) != hipSuccess) ||
      (P->queue_ok && (e = hipMalloc(&P->d_queue_order, sizeof(int) * P->n_pairs)) != hipSuccess) ||
      (P->queue_ok && (e = hipMalloc(&P->d_queue_counter, sizeof(int))) != hipSuccess)) {
    rheed_plan_destroy(P);
    return e == hipErrorOutOfMemory ? fail(RHEED_E_NOMEM, "plan_create: device allocation") : hip_fail(e, "hipMalloc");
  }
  if ((e = hipMemcpy(P->d_structs, P->hs.data(), sizeof(StructDev) * P->hs.size(), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(P->d_beams, P->beams.data(), sizeof(int) * P->beams.size(), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(P->d_pair_struct, P->pair_struct.data(), sizeof(int) * P->pair_struct.size(),
                     hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(P->d_bin_ptr, P->bin_ptr.data(), sizeof(int) * P->bin_ptr.size(), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(P->d_bin_jk, P->bin_jk.data(), sizeof(int) * P->bin_jk.size(), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (!P->atom_struct.empty() &&
       (e = hipMemcpy(P->d_atom_struct, P->atom_struct.data(), sizeof(long long) * P->atom_struct.size(),
                      hipMemcpyHostToDevice)) != hipSuccess) ||
      (P->split && (e = hipMemset(P->d_xch, 0, (size_t)XCH_STRIDE * n_small)) != hipSuccess) ||
      (P->d_small_pairs && (e = hipMemcpy(P->d_small_pairs, P->small_pairs.data(), sizeof(int) * n_small,
                                          hipMemcpyHostToDevice)) != hipSuccess) ||
      (P->d_xl_pairs && (e = hipMemcpy(P->d_xl_pairs, P->xl_pairs.data(), sizeof(int) * P->xl_pairs.size(),
                                        hipMemcpyHostToDevice)) != hipSuccess) ||
      (P->d_xxl_pairs && (e = hipMemcpy(P->d_xxl_pairs, P->xxl_pairs.data(), sizeof(int) * P->xxl_pairs.size(),
                                         hipMemcpyHostToDevice)) != hipSuccess) ||
      (P->d_large_pairs && (e = hipMemcpy(P->d_large_pairs, P->large_pairs.data(), sizeof(int) * n_large,
                                          hipMemcpyHostToDevice)) != hipSuccess) ||
      (P->d_large_plain && (e = hipMemcpy(P->d_large_plain, P->large_plain.data(), sizeof(int) * n_large,
                                          hipMemcpyHostToDevice)) != hipSuccess) ||
      (P->d_queue_order && (e = hipMemcpy(P->d_queue_order, P->queue_order.data(), sizeof(int) * P->n_pairs,
                                          hipMemcpyHostToDevice)) != hipSuccess) ||
      (e = hipDeviceSynchronize()) != hipSuccess) {
    rheed_plan_destroy(P);
    return hip_fail(e, "hipMemcpy");
  }
  {
    // rheed_potential_backward_noalloc's fixed array: its address on this
    // device, looked up here so that the entry point itself makes no setup call
    double* part = nullptr;
    if ((e = potential_bwd_scratch(&part)) != hipSuccess) {
      rheed_plan_destroy(P);
      return hip_fail(e, "hipGetSymbolAddress");
    }
  }
  *out = P;
  return RHEED_OK;
}

rheed_status rheed_plan_destroy(rheed_plan_t P) {
  if (!P) return RHEED_OK;
  if (P->d_structs) (void)hipFree(P->d_structs);
  if (P->d_beams) (void)hipFree(P->d_beams);
  if (P->d_pair_struct) (void)hipFree(P->d_pair_struct);
  if (P->d_atom_struct) (void)hipFree(P->d_atom_struct);
  if (P->d_bin_ptr) (void)hipFree(P->d_bin_ptr);
  if (P->d_bin_jk) (void)hipFree(P->d_bin_jk);
  if (P->d_pbwd) (void)hipFree(P->d_pbwd);
  if (P->d_xch) (void)hipFree(P->d_xch);
  if (P->d_small_pairs) (void)hipFree(P->d_small_pairs);
  if (P->d_large_pairs) (void)hipFree(P->d_large_pairs);
  if (P->d_large_plain) (void)hipFree(P->d_large_plain);
  if (P->d_lscratch) (void)hipFree(P->d_lscratch);
  if (P->d_xl_pairs) (void)hipFree(P->d_xl_pairs);
  if (P->d_xscratch) (void)hipFree(P->d_xscratch);
  if (P->d_xg_pair) (void)hipFree(P->d_xg_pair);
  if (P->d_xg_wg) (void)hipFree(P->d_xg_wg);
  if (P->d_xg_cnt) (void)hipFree(P->d_xg_cnt);
  if (P->d_xxl_pairs) (void)hipFree(P->d_xxl_pairs);
  if (P->d_xxg_pair) (void)hipFree(P->d_xxg_pair);
  if (P->d_xxg_wg) (void)hipFree(P->d_xxg_wg);
  if (P->d_xxg_cnt) (void)hipFree(P->d_xxg_cnt);
  if (P->d_queue_order) (void)hipFree(P->d_queue_order);
  if (P->d_queue_counter) (void)hipFree(P->d_queue_counter);
  delete P;
  return RHEED_OK;
}

rheed_status rheed_plan_get_info(rheed_plan_t P, rheed_plan_info* info) {
  if (!P || !info) return fail(RHEED_E_INVALID, "plan_get_info: null argument");
  info->n_struct = P->n_struct;
  info->n_pairs = P->n_pairs;
  info->max_beams = P->max_beams;
  info->nodes_per_slice = P->nodes_per_slice;
  info->table_elems = P->table_elems;
  info->n_atoms_total = P->n_atoms_total;
  info->fwd_workspace = P->fwd_ws;
  info->bwd_workspace = P->bwd_ws;
  info->split = P->split ? 1 : 0;
  info->split_max_pairs = P->split_max;
  info->large_pairs = (int32_t)P->large_pairs.size();
  info->large_slots = P->large_slots;
  info->bulk_workspace = (P->large_pairs.empty() && P->xl_pairs.empty() && P->xxl_pairs.empty()) ? bulk_extra(P) : 0;
  info->xl_pairs = (int32_t)P->xl_pairs.size();
  info->xl_slots = P->xl_slots;
  info->xl_group = P->xl_group;
  info->xxl_pairs = (int32_t)P->xxl_pairs.size();
  info->xxl_group = P->xxl_group;
  info->queue = (P->use_queue && P->queue_ok) ? 1 : 0;
  return RHEED_OK;
}

rheed_status rheed_plan_force_sync_failure(rheed_plan_t P, int32_t half) {
  if (!P || half < -1 || half > 1) return fail(RHEED_E_INVALID, "plan_force_sync_failure: half must be -1, 0 or 1");
  P->xch_give_up = half;
  return RHEED_OK;
}

rheed_status rheed_plan_table_offsets(rheed_plan_t P, int64_t* out) {
  if (!P || !out) return fail(RHEED_E_INVALID, "plan_table_offsets: null argument");
  for (size_t i = 0; i < P->table_off.size(); ++i) out[i] = P->table_off[i];
  return RHEED_OK;
}

rheed_status rheed_plan_atom_offsets(rheed_plan_t P, int64_t* out) {
  if (!P || !out) return fail(RHEED_E_INVALID, "plan_atom_offsets: null argument");
  for (size_t i = 0; i < P->atom_off.size(); ++i) out[i] = P->atom_off[i];
  return RHEED_OK;
}

rheed_status rheed_potential(rheed_plan_t P, const double* atoms, void* U_tables, void* stream) {
  if (!P || !U_tables || (P->n_atoms_total > 0 && !atoms)) return fail(RHEED_E_INVALID, "potential: null argument");
  PotArgs a{};
  a.structs = P->d_structs;
  a.atoms = atoms;
  a.U = static_cast<double2*>(U_tables);
  a.n_struct = P->n_struct;
  a.nodes_per_slice = P->nodes_per_slice;
  for (int c = 0; c < 12; ++c) a.cset[c] = P->cset[c];
  hipError_t e = launch_potential(a, P->max_table, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? RHEED_OK : hip_fail(e, "potential launch");
}

rheed_status rheed_potential_backward(rheed_plan_t P, const double* atoms, const void* dL_dU, double* dL_datoms,
                                      void* stream) {
  if (!P || !dL_dU || (P->n_atoms_total > 0 && (!atoms || !dL_datoms)))
    return fail(RHEED_E_INVALID, "potential_backward: null argument");
  if (P->n_atoms_total == 0) return RHEED_OK;
  PotBwdArgs a{};
  a.structs = P->d_structs;
  a.atoms = atoms;
  a.dU = static_cast<const double2*>(dL_dU);
  a.datoms = dL_datoms;
  a.partial = P->d_pbwd;
  a.nodes_per_slice = P->nodes_per_slice;
  for (int c = 0; c < 12; ++c) a.cset[c] = P->cset[c];
  hipError_t e = launch_potential_bwd(a, P->n_atoms_total, P->n_struct, P->d_atom_struct,
                                      static_cast<hipStream_t>(stream));
  return e == hipSuccess ? RHEED_OK : hip_fail(e, "potential_backward launch");
}

rheed_status rheed_potential_backward_noalloc(rheed_plan_t P, const double* atoms, const void* dL_dU,
                                              double* dL_datoms, void* stream) {
  if (!P || !dL_dU || (P->n_atoms_total > 0 && (!atoms || !dL_datoms)))
    return fail(RHEED_E_INVALID, "potential_backward_noalloc: null argument");
  if (P->n_atoms_total > RHEED_NOALLOC_MAX_ATOMS)
    return fail(RHEED_E_UNSUPPORTED, "potential_backward_noalloc: " + std::to_string(P->n_atoms_total) +
                                         " atoms exceed the fixed partial-sum array of " +
                                         std::to_string(RHEED_NOALLOC_MAX_ATOMS));
  if (P->n_atoms_total == 0) return RHEED_OK;
  double* part = nullptr;
  hipError_t e = potential_bwd_scratch(&part);
  if (e != hipSuccess) return hip_fail(e, "potential_backward_noalloc: hipGetSymbolAddress");
  PotBwdArgs a{};
  a.structs = P->d_structs;
  a.atoms = atoms;
  a.dU = static_cast<const double2*>(dL_dU);
  a.datoms = dL_datoms;
  a.partial = part;
  a.nodes_per_slice = P->nodes_per_slice;
  for (int c = 0; c < 12; ++c) a.cset[c] = P->cset[c];
  e = launch_potential_bwd(a, P->n_atoms_total, P->n_struct, P->d_atom_struct, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? RHEED_OK : hip_fail(e, "potential_backward_noalloc launch");
}

}  // extern "C"

namespace {

// rheed_forward with an optional bottom state [I; Y] per pair, an optional
// skip flag per pair (the bulk iteration's converged pairs) and, with a bottom
// state and a workspace, the option to keep only the final state.
rheed_status forward_impl(rheed_plan_t P, const void* U_tables, const double* angles, double* intensity, void* rho,
                          int32_t* pair_status, int32_t* n_rhst, void* workspace, size_t ws_bytes, void* stream,
                          const void* y_bottom, const int* skip, bool final_only = false) {
  if (!P || !U_tables || !angles || !intensity || !pair_status) return fail(RHEED_E_INVALID, "forward: null argument");
  const bool f32 = P->opts.stage_precision == RHEED_STAGES_FP32;
  if (workspace && ((P->splitting && !P->large_pairs.empty()) || f32 || !P->xxl_pairs.empty()))
    return fail(RHEED_E_UNSUPPORTED, "forward: keeping states for the adjoint needs FP64 stages, every structure "
                                     "to have N <= 256, and with a splitting stepper N <= 64");
  if (y_bottom && (!P->large_pairs.empty() || !P->xl_pairs.empty() || !P->xxl_pairs.empty()))
    return fail(RHEED_E_UNSUPPORTED, "forward: the bulk start needs every structure to have N <= 64");
  if (y_bottom && (P->splitting || f32))
    return fail(RHEED_E_UNSUPPORTED, "forward: the bulk start needs an RK stepper with FP64 stages");
  if (workspace && ws_bytes < P->fwd_ws)
    return fail(RHEED_E_INVALID, "forward: workspace of " + std::to_string(ws_bytes) + " bytes < " +
                                     std::to_string(P->fwd_ws));
  FwdArgs a{};
  a.y_bottom = static_cast<const double2*>(y_bottom);
  a.skip = skip;
  a.final_only = final_only ? 1 : 0;
  a.structs = P->d_structs;
  a.pair_struct = P->d_pair_struct;
  a.beams = P->d_beams;
  a.U = static_cast<const double2*>(U_tables);
  a.angles = angles;
  a.intensity = intensity;
  a.rho = static_cast<double2*>(rho);
  a.status = pair_status;
  a.nrhst = n_rhst;
  a.ws = static_cast<char*>(workspace);
  a.ck = P->ck;
  a.ld = P->max_beams;
  a.convention = (int)P->opts.convention;
  a.threshold = P->opts.rhst_threshold;
  a.xch_give_up = P->xch_give_up;
  a.sp = P->sp;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  if (P->use_queue && P->queue_ok && !workspace && !y_bottom && !skip) {
    // one persistent launch over the whole batch
    QueueArgs q{};
    q.large.f = a;
    q.large.f.pair_list = nullptr;
    q.large.f.n_pairs = P->n_pairs;
    q.large.scratch = P->d_lscratch;
    q.large.n_slots = P->scratch_slots;
    q.order = P->d_queue_order;
    q.counter = P->d_queue_counter;
    q.n = P->n_pairs;
    e = launch_forward_queue((int)P->opts.stepper, q, P->queue_grid, st);
    return e == hipSuccess ? RHEED_OK : hip_fail(e, "forward launch (one queue over the batch)");
  }
  if (!P->small_pairs.empty()) {
    a.pair_list = P->d_small_pairs;  // null when every pair is small
    a.n_pairs = (int)P->small_pairs.size();
    // kernel code: the method (0 RK4, 1 RK6, 2 a splitting method), plus 8 for FP32 stage products
    const int kcode = (P->splitting ? 2 : (int)P->opts.stepper) | (f32 ? 8 : 0);
    if (P->split) {
      a.xch = P->d_xch;
      e = launch_forward_split(kcode, a, st);
    } else {
      e = launch_forward(kcode, a, st);
    }
    if (e != hipSuccess) return hip_fail(e, "forward launch");
  }
  if (!P->large_pairs.empty()) {
    LargeArgs la{};
    la.f = a;
    la.f.pair_list = P->large_cost_order ? P->d_large_pairs : P->d_large_plain;
    la.f.n_pairs = (int)P->large_pairs.size();
    la.f.ck = P->ckl;
    la.f.xch = nullptr;
    la.scratch = P->d_lscratch;
    la.n_slots = P->large_slots;
    for (int q = 0; q < 3; ++q) la.sp_a[q] = P->sp_a[q];
    for (int q = 0; q < 4; ++q) la.sp_b[q] = P->sp_b[q];
    e = launch_forward_large((int)P->opts.stepper | (f32 ? 8 : 0), la, st);
    if (e != hipSuccess) return hip_fail(e, "forward launch (N > 64)");
  }
  if (!P->xl_pairs.empty()) {
    LargeArgs xa{};
    xa.f = a;
    xa.f.pair_list = P->d_xl_pairs;
    xa.f.n_pairs = (int)P->xl_pairs.size();
    xa.f.ck = P->ckx;
    xa.f.xch = nullptr;
    xa.scratch = P->d_xscratch;
    xa.n_slots = P->xl_slots;
    if (P->xl_group > 1) {
      XlGroup xg{};
      xg.pair_mem = P->d_xg_pair;
      xg.wg_mem = P->d_xg_wg;
      xg.counters = P->d_xg_cnt;
      xg.group = P->xl_group;
      e = launch_forward_xl_group((int)P->opts.stepper | (f32 ? 8 : 0), xa, xg, st);
    } else {
      e = launch_forward_xl((int)P->opts.stepper | (f32 ? 8 : 0), xa, st);
    }
    if (e != hipSuccess) return hip_fail(e, "forward launch (N > 128)");
  }
  if (!P->xxl_pairs.empty()) {
    LargeArgs xa{};
    xa.f = a;
    xa.f.ws = nullptr;
    xa.f.xch = nullptr;
    XlGroup xg{};
    xg.pair_mem = P->d_xxg_pair;
    xg.wg_mem = P->d_xxg_wg;
    xg.counters = P->d_xxg_cnt;
    xg.group = P->xxl_group;
    const int n_xxl = (int)P->xxl_pairs.size();
    for (int off = 0; off < n_xxl; off += P->xxl_per_launch) {  // launches on one stream run in order
      xa.f.pair_list = P->d_xxl_pairs + off;
      xa.f.n_pairs = std::min(P->xxl_per_launch, n_xxl - off);
      e = launch_forward_xxl_group((int)P->opts.stepper, xa, xg, st);
      if (e != hipSuccess) return hip_fail(e, "forward launch (N > 256)");
    }
  }
  return RHEED_OK;
}

}  // namespace

extern "C" {

rheed_status rheed_forward(rheed_plan_t P, const void* U_tables, const double* angles, double* intensity, void* rho,
                           int32_t* pair_status, int32_t* n_rhst, void* workspace, size_t ws_bytes, void* stream) {
  return forward_impl(P, U_tables, angles, intensity, rho, pair_status, n_rhst, workspace, ws_bytes, stream,
                      nullptr, nullptr);
}

rheed_status rheed_forward_bulk(rheed_plan_t P, const void* U_tables, const double* angles, const void* y_bottom,
                                double* intensity, void* rho, int32_t* pair_status, int32_t* n_rhst, void* workspace,
                                size_t ws_bytes, void* stream) {
  if (!P || !y_bottom) return fail(RHEED_E_INVALID, "forward_bulk: null argument");
  if (!P->large_pairs.empty() || !P->xl_pairs.empty() || !P->xxl_pairs.empty() || P->splitting ||
      P->opts.stage_precision != RHEED_STAGES_FP64)
    return fail(RHEED_E_UNSUPPORTED, "forward_bulk: needs an RK stepper with FP64 stages and every structure to have N <= 64");
  return forward_impl(P, U_tables, angles, intensity, rho, pair_status, n_rhst, workspace, ws_bytes, stream,
                      y_bottom, nullptr);
}

rheed_status rheed_bulk_reflection(rheed_plan_t P, const void* U_tables, const double* angles, double tol,
                                   int32_t max_layers, void* y_bulk, void* r_bulk, int32_t* layers,
                                   int32_t* pair_status, void* workspace, size_t ws_bytes, void* stream) {
  if (!P || !U_tables || !angles || !y_bulk || !r_bulk || !layers || !pair_status || !workspace)
    return fail(RHEED_E_INVALID, "bulk_reflection: null argument");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(RHEED_E_INVALID, "bulk_reflection: tol must be finite and >= 0");
  if (max_layers < 1) return fail(RHEED_E_INVALID, "bulk_reflection: max_layers must be >= 1");
  if (!P->large_pairs.empty() || !P->xl_pairs.empty() || !P->xxl_pairs.empty() || P->splitting ||
      P->opts.stage_precision != RHEED_STAGES_FP64)
    return fail(RHEED_E_UNSUPPORTED, "bulk_reflection: needs an RK stepper with FP64 stages and every structure to have N <= 64");
  const size_t need = P->fwd_ws + bulk_extra(P);
  if (ws_bytes < need)
    return fail(RHEED_E_INVALID, "bulk_reflection: workspace of " + std::to_string(ws_bytes) + " bytes < " +
                                     std::to_string(need));
  const size_t np = (size_t)P->n_pairs, m = (size_t)P->max_beams;
  char* base = static_cast<char*>(workspace) + P->fwd_ws;
  double* inten = reinterpret_cast<double*>(base);
  base += align256(np * m * 8);
  int* done = reinterpret_cast<int*>(base);
  base += align256(np * 4);
  int* fstat = reinterpret_cast<int*>(base);
  hipStream_t st = static_cast<hipStream_t>(stream);
  BulkArgs b{};
  b.structs = P->d_structs;
  b.pair_struct = P->d_pair_struct;
  b.beams = P->d_beams;
  b.angles = angles;
  b.ws = static_cast<const char*>(workspace);
  b.ck = P->ck;
  b.y = static_cast<double2*>(y_bulk);
  b.r = static_cast<double2*>(r_bulk);
  b.done = done;
  b.layers = layers;
  b.status = pair_status;
  b.fstatus = fstat;
  b.ld = P->max_beams;
  b.n_pairs = P->n_pairs;
  b.tol = tol;
  hipError_t e = launch_bulk_init(b, st);
  if (e != hipSuccess) return hip_fail(e, "bulk_reflection: init launch");
  std::vector<int> host_done(np);
  for (int it = 1; it <= max_layers; ++it) {
    // one unit layer from [I; Y] for every pair still iterating, then Y and R at its top
    rheed_status s = forward_impl(P, U_tables, angles, inten, nullptr, fstat, nullptr, workspace, P->fwd_ws, stream,
                                  y_bulk, done, true);
    if (s != RHEED_OK) return s;
    b.iter = it;
    e = launch_bulk_update(b, st);
    if (e != hipSuccess) return hip_fail(e, "bulk_reflection: update launch");
    e = hipMemcpyAsync(host_done.data(), done, np * sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "bulk_reflection: reading the convergence flags");
    bool all = true;
    for (size_t q = 0; q < np && all; ++q) all = host_done[q] != 0;
    if (all) break;
  }
  return RHEED_OK;
}

rheed_status rheed_autotune(rheed_plan_t P, const void* U_tables, const double* angles, double* intensity,
                            int32_t* pair_status, int32_t reps, void* stream, rheed_tune_report* report) {
  if (!P || !U_tables || !angles || !intensity || !pair_status || reps < 1 || reps > 1000)
    return fail(RHEED_E_INVALID, "autotune: null argument or reps outside [1, 1000]");
  // candidates: one persistent launch over the batch (when it mixes N <= 64
  // and N > 64), and two launches with the N <= 64 layouts the plan allows
  // (split needs its exchange blocks, allocated when the batch fits) x the
  // N > 64 pair orders
  struct Cand {
    bool split, cost_order, queue;
  };
  std::vector<Cand> cand;
  const bool has_small = !P->small_pairs.empty(), has_large = !P->large_pairs.empty();
  if (P->queue_ok) cand.push_back({false, true, true});
  std::vector<bool> layouts;
  if (!has_small) layouts = {P->split};
  else if (P->d_xch && P->opts.layout == RHEED_LAYOUT_AUTO) layouts = {true, false};
  else layouts = {P->split};
  std::vector<bool> orders = has_large ? std::vector<bool>{true, false} : std::vector<bool>{P->large_cost_order};
  for (bool l : layouts)
    for (bool o : orders) cand.push_back({l, o, false});
  if ((int)cand.size() > RHEED_TUNE_MAX) cand.resize(RHEED_TUNE_MAX);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_fail(e, "autotune: hipEventCreate");
  }
  const bool keep_split = P->split, keep_order = P->large_cost_order, keep_queue = P->use_queue;
  std::vector<float> ms(cand.size(), 0.0f);
  rheed_status rs = RHEED_OK;
  for (size_t c = 0; c < cand.size() && rs == RHEED_OK; ++c) {
    P->split = cand[c].split;
    P->large_cost_order = cand[c].cost_order;
    P->use_queue = cand[c].queue;
    rs = rheed_forward(P, U_tables, angles, intensity, nullptr, pair_status, nullptr, nullptr, 0, stream);  // untimed
    if (rs != RHEED_OK) break;
    if ((e = hipEventRecord(e0, st)) != hipSuccess) { rs = hip_fail(e, "autotune: hipEventRecord"); break; }
    for (int r = 0; r < reps && rs == RHEED_OK; ++r)
      rs = rheed_forward(P, U_tables, angles, intensity, nullptr, pair_status, nullptr, nullptr, 0, stream);
    if (rs != RHEED_OK) break;
    if ((e = hipEventRecord(e1, st)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
        (e = hipEventElapsedTime(&ms[c], e0, e1)) != hipSuccess) {
      rs = hip_fail(e, "autotune: timing");
      break;
    }
    ms[c] /= (float)reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rs != RHEED_OK) {
    P->split = keep_split;
    P->large_cost_order = keep_order;
    P->use_queue = keep_queue;
    return rs;
  }
  size_t best = 0;
  for (size_t c = 1; c < cand.size(); ++c)
    if (ms[c] < ms[best]) best = c;
  P->split = cand[best].split;
  P->large_cost_order = cand[best].cost_order;
  P->use_queue = cand[best].queue;
  if (report) {
    *report = rheed_tune_report{};
    report->n_candidates = (int32_t)cand.size();
    report->chosen = (int32_t)best;
    for (size_t c = 0; c < cand.size(); ++c) {
      report->split[c] = cand[c].split ? 1 : 0;
      report->large_cost_order[c] = cand[c].cost_order ? 1 : 0;
      report->queue[c] = cand[c].queue ? 1 : 0;
      report->ms[c] = ms[c];
    }
  }
  return RHEED_OK;
}

rheed_status rheed_backward(rheed_plan_t P, const void* U_tables, const double* angles, const double* dL_dI,
                            void* dL_dU, void* workspace, size_t ws_bytes, void* stream) {
  if (!P || !U_tables || !angles || !dL_dI || !dL_dU || !workspace)
    return fail(RHEED_E_INVALID, "backward: null argument");
  if ((P->splitting && !P->large_pairs.empty()) || P->opts.stage_precision != RHEED_STAGES_FP64 ||
      !P->xxl_pairs.empty())
    return fail(RHEED_E_UNSUPPORTED, "backward: the adjoint needs FP64 stages, every structure to have N <= 256, "
                                     "and with a splitting stepper N <= 64");
  if (ws_bytes < P->fwd_ws + P->bwd_ws)
    return fail(RHEED_E_INVALID, "backward: workspace of " + std::to_string(ws_bytes) + " bytes < " +
                                     std::to_string(P->fwd_ws + P->bwd_ws));
  BwdArgs a{};
  a.structs = P->d_structs;
  a.pair_struct = P->d_pair_struct;
  a.beams = P->d_beams;
  a.U = static_cast<const double2*>(U_tables);
  a.angles = angles;
  a.dLdI = dL_dI;
  a.ws = static_cast<const char*>(workspace);
  a.ck = P->ck;
  a.gbuf = reinterpret_cast<double2*>(static_cast<char*>(workspace) + P->fwd_ws);
  a.g_pair_stride = P->g_pair_stride;
  if (P->ck.every > 1) {
    a.xs = reinterpret_cast<double2*>(static_cast<char*>(workspace) + P->fwd_ws + P->xs_off);
    a.xs_stride = (long long)P->ck.every * (!P->xl_pairs.empty() ? NX : !P->large_pairs.empty() ? NL : NP);
  }
  a.ld = P->max_beams;
  a.convention = (int)P->opts.convention;
  a.sp = P->sp;
  const int bcode = P->splitting ? 2 : (int)P->opts.stepper;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  if (!P->small_pairs.empty()) {  // N <= 64: the 64-wide state layout
    a.pair_list = P->d_small_pairs;  // null when every pair is small
    a.n_pairs = (int)P->small_pairs.size();
    e = launch_backward(bcode, NP, a, st);
    if (e != hipSuccess) return hip_fail(e, "backward launch");
  }
  if (!P->large_pairs.empty()) {  // 64 < N <= 128: the 128-wide layout
    BwdArgs b = a;
    b.ck = P->ckl;
    b.pair_list = P->d_large_plain;
    b.n_pairs = (int)P->large_pairs.size();
    e = launch_backward((int)P->opts.stepper, NL, b, st);
    if (e != hipSuccess) return hip_fail(e, "backward launch (N > 64)");
  }
  if (!P->xl_pairs.empty()) {  // 128 < N <= 256: the 256-wide layout
    BwdArgs b = a;
    b.ck = P->ckx;
    b.pair_list = P->d_xl_pairs;
    b.n_pairs = (int)P->xl_pairs.size();
    e = launch_backward((int)P->opts.stepper, NX, b, st);
    if (e != hipSuccess) return hip_fail(e, "backward launch (N > 128)");
  }
  // stages that use each node of a slice: node offsets of the stages in
  // {0, 1/2} (RK4) or {0, 1/3, 1/2, 2/3} (RK6); offset nps is the next slice's 0
  GradArgs g{};
  g.structs = P->d_structs;
  g.gbuf = a.gbuf;
  g.g_pair_stride = a.g_pair_stride;
  g.bin_ptr = P->d_bin_ptr;
  g.bin_jk = P->d_bin_jk;
  g.dU = static_cast<double2*>(dL_dU);
  const bool rk4 = P->opts.stepper == RHEED_RK4;
  static const int node4[4] = {0, 1, 1, 2}, node6[7] = {0, 1, 3, 1, 2, 2, 4};
  g.stages = rk4 ? 4 : 7;
  g.nps = P->nodes_per_slice;
  const int* node = rk4 ? node4 : node6;
  if (P->splitting) {
    // the kicks kept per slice (the BAB method's first one carries the
    // previous slice's last), each at its node of the slice; the BAB final
    // kick is kick 0 of one more slice (node L nps)
    g.stages = P->sp.form == 0 ? P->sp.kicks - 1 : P->sp.kicks;
    g.last_extra = P->sp.form == 0 ? 1 : 0;
    node = P->sp.node;
  }
  for (int r = 0; r < g.stages; ++r) {
    const int res = node[r] % g.nps, di = node[r] / g.nps;  // node i nps + node[r] = (i + di) nps + res
    if (g.n_contrib[res] >= 2) return fail(RHEED_E_UNSUPPORTED, "backward: more than two kicks at one node");
    const int t = g.n_contrib[res]++;
    g.contrib_di[res][t] = -di;
    g.contrib_r[res][t] = r;
  }
  e = launch_grad_assemble(g, P->n_struct, P->max_nodes, !P->small_pairs.empty(), !P->large_pairs.empty(),
                           !P->xl_pairs.empty(), st);
  return e == hipSuccess ? RHEED_OK : hip_fail(e, "gradient assembly launch");
}

rheed_status rheed_rfactor(int32_t n_pairs, int32_t ld, const double* intensity, const double* target, double* loss,
                           double* dL_dI, void* stream) {
  if (n_pairs < 1 || ld < 1 || !intensity || !target || (!loss && !dL_dI))
    return fail(RHEED_E_INVALID, "rfactor: bad argument");
  hipError_t e = launch_rfactor(n_pairs, ld, intensity, target, loss, dL_dI, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? RHEED_OK : hip_fail(e, "rfactor launch");
}

}  // extern "C"
