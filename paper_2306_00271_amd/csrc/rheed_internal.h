// Internal descriptors shared by the host API and the HIP kernels of librheed.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rheed {

constexpr int NP = 64;          // padded beam count of the N <= 64 kernels
constexpr int MAXBOX = 300;     // rod-difference entries per node table row in LDS

// Device-side copy of one structure.
struct StructDev {
  int n_beams, n_slices, hd, kd;
  int box, n_nodes, n_atoms, beam_off;
  int pair_off, n_angles, bin_ptr_off, bin_jk_off;  // bins: (j,k) pairs of each rod difference
  double h, thickness, gamma, pad2;
  double recip[4];
  long long table_off;   // complex elements
  long long atom_off;    // atoms
  double scat_a[4], scat_b[4];
  double pref_re, pref_im;  // kappa * s * (charge - i alpha) / A  (volts -> 1/A^2 per unit cell area)
};

// Per-pair storage kept by the forward pass for the adjoint: the state (c, c')
// at the start of every slice and after the last one, T = Q^{-1} of every
// slice that was followed by a right-hand-side transformation, and one byte
// per slice telling whether that transformation was applied.  Matrices are
// padded to the kernel's beam count W (NP = 64 for N <= 64, 128 above),
// row major with row stride W; a plan with both kinds keeps two layouts with
// one pair stride.
struct CkptLayout {
  long long pair_stride;   // bytes per pair
  long long state_bytes;   // one state: 2 * W * W complex
  int every;               // slices between stored states (1: every slice)
  int max_ckpt;            // stored states per pair, including the final state
  long long q_off;         // byte offset of the T slots (one per slice)
  long long r_off;         // byte offset of the R slots (one per slice) when every > 1, else 0
  long long flags_off;     // byte offset of the decision bytes
  long long binv_off;      // W = 128 only: byte offset of B^{-1} of the reflection solve, else 0
};

// A splitting method (Sec. 3.4) for the one-workgroup kernel: kicks
// c' -= h b_r (U(tau_r) + Gamma^2) c and drifts c += h a_r c'.  BAB: kicks
// b_0 .. b_s with drifts a_0 .. a_{s-1} between them, the last kick at the
// slice end (merged into the next slice's first); ABA: drifts a_0 .. a_s
// with kicks b_0 .. b_{s-1} between them.  Kick r uses the table of node
// i nps + node[r] of slice i (node[r] = nps: the next slice's first node).
constexpr int MAX_KICKS = 10;
struct SplitSteps {
  int form;                  // 0: BAB, 1: ABA
  int nps;                   // node tables per slice (at most 12)
  int kicks;                 // kicks per slice
  int pad;
  double a[MAX_KICKS + 1];
  double b[MAX_KICKS + 1];
  int node[MAX_KICKS + 1];
};

struct FwdArgs {
  const StructDev* structs;
  const int* pair_struct;
  const int* pair_list;      // pair of each launch slot (n_pairs entries), or null: slot = pair
  const int* beams;          // packed [.][2]
  const double2* U;          // all tables
  const double* angles;      // [P][2]
  double* intensity;         // [P][ld]
  double2* rho;              // [P][ld] or null
  int* status;               // [P]
  int* nrhst;                // [P] or null
  char* ws;                  // checkpoints or null
  CkptLayout ck;
  int ld;
  int convention;
  int n_pairs;               // pairs of this launch
  int xch_give_up;           // split launches: the half (0, 1) whose first wait fails at once; group launches:
                             // the workgroup of each group that starts as if it had given up; -1 normally
  double threshold;
  // split launches (two workgroups per pair): per-pair exchange blocks
  char* xch;
  // bottom condition of a bulk below the slab: the state starts as [I; Y],
  // Y of pair p at y_bottom + p ld ld, row major (null: the vacuum, [I; i Gamma])
  const double2* y_bottom;
  const int* skip;           // [P] pairs with skip[p] != 0 are not run (or null)
  int final_only;            // with ws and a bulk start: keep only the final state (no adjoint follows)
  int pad2;
  SplitSteps sp;             // splitting steppers on the one-workgroup kernel
};

// A pair whose final reflection solve has ||B||_inf ||B^{-1} e_1||_inf above
// this (B = Gamma Q - iP, a lower bound of cond_inf(B)) is reported
// RHEED_PAIR_BREAKDOWN: its amplitudes would carry no correct digit.
constexpr double BREAKDOWN_COND = 1.0e14;

// Gamma_j from g2 = Gamma_j^2 (Sec. 2.1): sqrt(g2) for open beams, -i sqrt(-g2)
// for evanescent ones.
__device__ inline double2 gamma_of(double g2) {
  return g2 >= 0.0 ? make_double2(sqrt(g2), 0.0) : make_double2(0.0, -sqrt(-g2));
}

// Exchange block of one pair in a split launch (bytes): two 64-bit counters,
// the launch number and the two halves' failure words (the launch number in
// which the half gave up a wait), per half and parity the badness partials [2][NP]
// doubles, and per half and parity the half's [Q; P] columns, [2][NP][32]
// complex.
constexpr long long XCH_XI = 256;
constexpr long long XCH_BIG = XCH_XI + 2 * 2 * 2 * NP * 8;
constexpr long long XCH_HALF = 2LL * NP * 32 * 16;
constexpr long long XCH_STRIDE = XCH_BIG + 2 * 2 * XCH_HALF;

struct PotArgs {
  const StructDev* structs;
  const double* atoms;   // [n_atoms_total][3]
  double2* U;            // tables
  int n_struct;
  int nodes_per_slice;
  double cset[12];       // node positions of a slice, in units of h from its start
};

constexpr int PBWD_CHUNKS = 64;  // partial sums per atom in the potential adjoint
// atoms the fixed partial-sum array of rheed_potential_backward_noalloc holds
// (PBWD_STATIC_ATOMS x PBWD_CHUNKS x 3 doubles = 6 MiB per device)
constexpr long long PBWD_STATIC_ATOMS = 4096;

struct PotBwdArgs {
  const StructDev* structs;
  const double* atoms;
  const double2* dU;     // dL/dRe(u) + i dL/dIm(u)
  double* datoms;        // [n_atoms_total][3]
  double* partial;       // [n_atoms_total][PBWD_CHUNKS][3] (plan-owned)
  int nodes_per_slice;
  double cset[12];
};

struct BwdArgs {
  const StructDev* structs;
  const int* pair_struct;
  const int* pair_list;      // pair of each launch slot (n_pairs entries), or null: slot = pair
  const int* beams;
  const double2* U;
  const double* angles;
  const double* dLdI;        // [P][ld]
  const char* ws;            // forward workspace
  CkptLayout ck;
  double2* gbuf;             // stage buffer: per pair [slice][stage][v | g][W]
  long long g_pair_stride;   // elements per pair
  double2* xs;               // ck.every > 1: per pair [ck.every][W], x of the segment's transformed states
  long long xs_stride;       // elements per pair
  int ld;
  int convention;
  int n_pairs;
  int pad;
  SplitSteps sp;             // the splitting stepper's kicks and drifts (N <= 64)
};

// Stages (RK) or kicks (splitting) that use node n = i * nps + res:
// (slice i + contrib_di, stage or kick contrib_r); with last_extra the stage
// buffer holds one more slice (the BAB method's final kick, node L nps).
struct GradArgs {
  const StructDev* structs;
  const double2* gbuf;
  long long g_pair_stride;
  const int* bin_ptr;        // per structure: box + 1 offsets into bin_jk
  const int* bin_jk;         // j * W + k (W = 64 for N <= 64, else 128)
  double2* dU;               // all tables
  int stages;
  int nps;
  int last_extra;
  int pad;
  int n_contrib[12];
  int contrib_di[12][2];
  int contrib_r[12][2];
};

// The bulk layer: from the final states a forward pass over one unit layer
// kept, the normalised state [I; Y] and the reflection matrix at the layer's
// top, and the convergence test of the stack.
struct BulkArgs {
  const StructDev* structs;
  const int* pair_struct;
  const int* beams;
  const double* angles;
  const char* ws;            // forward workspace holding each pair's final state
  CkptLayout ck;
  double2* y;                // [P][ld][ld]: bottom state of this layer in, top state out
  double2* r;                // [P][ld][ld]: reflection matrix below this layer in, at its top out
  int* done;                 // [P]: 1 once converged or failed
  int* layers;               // [P]: unit layers at convergence, -1 until then
  int* status;               // [P]: RHEED_PAIR_* of the iteration
  const int* fstatus;        // [P]: the forward pass's status for this layer
  int ld;
  int n_pairs;
  int iter;                  // layers applied including this one
  int pad;
  double tol;
};

hipError_t launch_forward(int stepper, const FwdArgs& a, hipStream_t stream);
hipError_t launch_bulk_update(const BulkArgs& a, hipStream_t stream);
hipError_t launch_bulk_init(const BulkArgs& a, hipStream_t stream);  // vacuum start, flags cleared
hipError_t launch_forward_split(int stepper, const FwdArgs& a, hipStream_t stream);
int forward_split_max_pairs(int device);  // pairs a split launch can hold at once (0: not available)
// width: the state layout of the launch's pairs, 64 (N <= 64), 128 (N <= 128) or 256
hipError_t launch_backward(int stepper, int width, const BwdArgs& a, hipStream_t stream);
// narrow / wide / xl: launch the assembly for the structures with N <= 64 /
// 64 < N <= 128 / 128 < N <= 256
hipError_t launch_grad_assemble(const GradArgs& a, int n_struct, int max_nodes, bool narrow, bool wide, bool xl,
                                hipStream_t stream);
hipError_t launch_potential(const PotArgs& a, long long max_elems, hipStream_t stream);
hipError_t launch_potential_bwd(const PotBwdArgs& a, long long n_atoms_total, int n_struct,
                                const long long* atom_struct, hipStream_t stream);
// Device address of the fixed partial-sum array on the current device
// (looked up once per device; the lookup allocates nothing).
hipError_t potential_bwd_scratch(double** out);
hipError_t launch_rfactor(int n_pairs, int ld, const double* I, const double* t, double* loss, double* dI,
                          hipStream_t stream);

}  // namespace rheed
