// Internal descriptors of the 64 < N <= 128 forward path.
#pragma once
#include "rheed_internal.h"

namespace rheed {

constexpr int NL = 128;         // padded beam count of the large kernel
constexpr int MAXBOXL = 1024;   // rod-difference entries per node table row in its LDS

// Device memory of one resident workgroup of the large kernel: c and c' of
// the pair it is running ([NL][NL] complex each, row major) and the column
// operations of its last elimination ([NL][NL] complex: multipliers of step k
// in row k).
constexpr long long LSLOT_C = 0;
constexpr long long LSLOT_D = (long long)NL * NL * 16;
constexpr long long LSLOT_F = 2LL * NL * NL * 16;
constexpr long long LSLOT_BYTES = 3LL * NL * NL * 16;

constexpr int NX = 256;         // padded beam count of the kernel for 128 < N <= 256
constexpr int MAXBOXX = 1536;   // rod-difference entries per node table row of that kernel

// Device memory of one resident workgroup of the kernel for 128 < N <= 256:
// c and c' ([NX][NX] complex), the multipliers of its last elimination
// ([NX][NX]) and the stage products of one column block ([6][NX][16]).
constexpr long long XSLOT_C = 0;
constexpr long long XSLOT_D = (long long)NX * NX * 16;
constexpr long long XSLOT_F = 2LL * NX * NX * 16;
constexpr long long XSLOT_G = 3LL * NX * NX * 16;
constexpr long long XSLOT_BYTES = XSLOT_G + 6LL * NX * 16 * 16;

struct LargeArgs {
  FwdArgs f;       // f.pair_list / f.n_pairs: the pairs this kernel runs
  char* scratch;   // n_slots * LSLOT_BYTES, plan-owned
  int n_slots;     // workgroups of the launch (each loops over pairs)
  int pad;
  // splitting stepper: drift weights a_1..a_3 and kick weights b_1..b_4
  double sp_a[3];
  double sp_b[4];
};

hipError_t launch_forward_large(int stepper, const LargeArgs& a, hipStream_t stream);
int forward_large_slots(int device);  // resident workgroups of the large kernel on the device
// 128 < N <= 256 (RK steppers, forward only): scratch holds n_slots * XSLOT_BYTES
hipError_t launch_forward_xl(int stepper, const LargeArgs& a, hipStream_t stream);
int forward_xl_slots(int device);

// Group launch of the same kernel for small batches: `group` workgroups per
// pair share the pair's state.  Per pair: c, c', the multipliers and the
// pivot list (XG_PAIR_BYTES); per workgroup: the stage products of one
// column block and two buffers of row-sum partials (XG_WG_BYTES); per pair
// XG_CTR_WORDS counter words (barrier count, failure word, and the progress
// words of the elimination pipeline), cleared by the launch.
constexpr long long XG_STAGE_BYTES = 6LL * NX * 16 * 16;
constexpr int XG_CTR_WORDS = 64;  // per pair: [0] barrier count, [1] failure word, [2] blocks recorded,
                                  // [3 + g] blocks applied by workgroup g (g < 61)
constexpr long long XG_PAIR_BYTES = XSLOT_G + 4LL * NX;
constexpr long long XG_WG_BYTES = XG_STAGE_BYTES + 2LL * 2 * NX * 8;
struct XlGroup {
  char* pair_mem;
  char* wg_mem;
  unsigned* counters;
  int group;
  int pad;
};
hipError_t launch_forward_xl_group(int stepper, const LargeArgs& a, const XlGroup& x, hipStream_t stream);
int forward_xl_group_max_workgroups(int device);  // co-resident workgroups of a group launch (0: none)

// 256 < N <= 576 (RK steppers, forward only), group launch only: a pair's
// c, c', multipliers and pivot list (XXG_PAIR_BYTES); per workgroup the 7
// stage products and the stage input of one column block and two buffers
// of row-sum partials (XXG_WG_BYTES); XG_CTR_WORDS counter words per pair.
constexpr int NXX = 576;        // padded beam count of the kernel for 256 < N <= 576
constexpr int MAXBOXXX = 4096;  // rod-difference entries per node table row of that kernel
constexpr long long XXG_C = 0;
constexpr long long XXG_D = (long long)NXX * NXX * 16;
constexpr long long XXG_F = 2LL * NXX * NXX * 16;
constexpr long long XXG_PIV = 3LL * NXX * NXX * 16;
constexpr long long XXG_PAIR_BYTES = XXG_PIV + 4LL * NXX;
constexpr long long XXG_STAGE_BYTES = 8LL * NXX * 16 * 16;  // G_0 .. G_6 and X of a block
constexpr long long XXG_WG_BYTES = XXG_STAGE_BYTES + 2LL * 2 * NXX * 8;
hipError_t launch_forward_xxl_group(int stepper, const LargeArgs& a, const XlGroup& x, hipStream_t stream);
int forward_xxl_group_max_workgroups(int device);  // co-resident workgroups of its launch (0: none)

// One persistent launch over a batch of pairs with N <= 64 and N > 64
// (forward_queue_kernel): workgroups take pairs in the order of `order`
// from a counter in device memory; the N <= 64 pairs run the one-workgroup
// path, the others the large path in the workgroup's state slot.
struct QueueArgs {
  LargeArgs large;   // large.f: the forward arguments of the batch (RK, vacuum start, no state saving);
                     // large.scratch / n_slots: one state slot per workgroup
  const int* order;  // [n] pairs, dearest first
  int* counter;      // device int, set to 0 by the launch before the workgroups start
  int n;
  int pad;
};
hipError_t launch_forward_queue(int stepper, const QueueArgs& q, int grid, hipStream_t stream);
int forward_queue_slots(int device);  // resident workgroups of forward_queue_kernel on the device

}  // namespace rheed
