// Internal descriptors shared by the host API and the HIP kernels of librheed.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rheed {

constexpr int NP = 64;          // padded beam count of the N <= 64 kernels
constexpr int NWAVES = 4;       // waves per workgroup of the propagation kernels (one per SIMD)
constexpr int NTHREADS = NWAVES * 64;
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
// at the start of every slice and after the last one, the upper block Q of
// every slice that was followed by a right-hand-side transformation (before
// it), and one byte per slice telling whether that transformation was applied.
struct CkptLayout {
  long long pair_stride;   // bytes per pair
  long long state_bytes;   // one state: 2 * NP * NP complex
  int every;               // slices between stored states (1: every slice)
  int max_ckpt;            // stored states per pair, including the final state
  long long q_off;         // byte offset of the Q slots (one per slice)
  long long flags_off;     // byte offset of the decision bytes
};

struct FwdArgs {
  const StructDev* structs;
  const int* pair_struct;
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
  int n_pairs;
  int pad;
  double threshold;
};

struct PotArgs {
  const StructDev* structs;
  const double* atoms;   // [n_atoms_total][3]
  double2* U;            // tables
  int n_struct;
  int nodes_per_slice;
  double cset[4];        // distinct RK node fractions in [0, 1)
};

struct PotBwdArgs {
  const StructDev* structs;
  const double* atoms;
  const double2* dU;     // dL/dRe(u) + i dL/dIm(u)
  double* datoms;        // [n_atoms_total][3]
  int nodes_per_slice;
  double cset[4];
};

struct BwdArgs {
  const StructDev* structs;
  const int* pair_struct;
  const int* beams;
  const double2* U;
  const double* angles;
  const double* dLdI;        // [P][ld]
  const char* ws;            // forward workspace
  CkptLayout ck;
  double2* ubar;             // per-pair dL/dU tables, stride ubar_stride elements
  long long ubar_stride;
  const int* bin_ptr;        // per structure: box + 1 offsets into bin_jk
  const int* bin_jk;         // j * NP + k
  int ld;
  int convention;
  int n_pairs;
  int stages;
  int nodes_per_slice;
  int stage_node[7];         // node offset of each stage inside its slice (nodes_per_slice = next slice)
  double A[7][7];
  double b[7];
};

struct ReduceArgs {
  const StructDev* structs;
  const double2* ubar;
  long long ubar_stride;
  double2* dU;               // all tables
};

hipError_t launch_forward(int stepper, const FwdArgs& a, hipStream_t stream);
hipError_t launch_backward(const BwdArgs& a, hipStream_t stream);
hipError_t launch_reduce_ubar(const ReduceArgs& a, int n_struct, long long max_table, hipStream_t stream);
hipError_t launch_potential(const PotArgs& a, long long max_elems, hipStream_t stream);
hipError_t launch_potential_bwd(const PotBwdArgs& a, long long n_atoms_total, int n_struct,
                                const long long* atom_struct, hipStream_t stream);
hipError_t launch_rfactor(int n_pairs, int ld, const double* I, const double* t, double* loss, double* dI,
                          hipStream_t stream);

}  // namespace rheed
