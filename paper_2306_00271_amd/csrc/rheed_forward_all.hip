// The translation unit of every forward kernel: the kernels for N <= 64
// (rheed_forward.hip), the kernel for 64 < N <= 128
// (rheed_forward_large.hip), those for 128 < N <= 256 and 256 < N <= 576
// (rheed_forward_xl.hip, rheed_forward_xxl.hip), and forward_queue_kernel,
// one persistent launch over a batch that mixes N <= 64 and 64 < N <= 128
// (the batching of Sec. 3.5 over (structure, angle) pairs, here of uneven
// beam counts).  They are one unit so that the LDS of the two pair
// paths is one allocation: a workgroup of forward_queue_kernel runs pairs of
// either kind one after another in the same LDS.
#include "rheed_forward.hip"
#include "rheed_forward_large.hip"
#include "rheed_forward_xl.hip"
#include "rheed_forward_xxl.hip"

namespace rheed {

union ForwardLds {
  Lds small;
  LLds large;
};
__shared__ ForwardLds forward_lds;

__device__ Lds& fwd_lds_ref() { return forward_lds.small; }
namespace {
__device__ LLds& large_lds_ref() { return forward_lds.large; }
}  // namespace

namespace {

static_assert(FT == LT, "the two pair paths run on workgroups of the same size");

// Persistent workgroups take pairs from a shared counter in the order of
// q.order (dearest first) until the batch is done; each runs the pair on the
// path of its beam count.  No workgroup waits for another.
template <int STEPPER>
__global__ __launch_bounds__(LT, 1) void forward_queue_kernel(QueueArgs q) {
  __shared__ int next;
  char* slot = q.large.scratch + (long long)blockIdx.x * LSLOT_BYTES;
#pragma unroll 1
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(q.counter, 1);
    __syncthreads();
    const int k = next;
    __syncthreads();
    if (k >= q.n) break;
    const int p = q.order[k];
    if (q.large.f.structs[q.large.f.pair_struct[p]].n_beams <= NP)
      small_pair<STEPPER, false>(q.large.f, p);
    else
      run_pair<STEPPER, false>(q.large, p, slot);
    __syncthreads();  // LDS is reused by the next pair
  }
}

__global__ void queue_reset_kernel(int* counter) {
  if (threadIdx.x == 0) *counter = 0;
}

}  // namespace

hipError_t launch_forward_queue(int stepper, const QueueArgs& q, int grid, hipStream_t stream) {
  if (q.n < 1) return hipSuccess;
  if (grid < 1 || grid > q.large.n_slots || (stepper != 0 && stepper != 1)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(64), 0, stream, q.counter);
  if (stepper == 0)
    hipLaunchKernelGGL(forward_queue_kernel<0>, dim3(grid), dim3(LT), 0, stream, q);
  else
    hipLaunchKernelGGL(forward_queue_kernel<1>, dim3(grid), dim3(LT), 0, stream, q);
  return hipGetLastError();
}

int forward_queue_slots(int device) {
  int cus = 0, p0 = 0, p1 = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&p0, forward_queue_kernel<0>, LT, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&p1, forward_queue_kernel<1>, LT, 0) != hipSuccess)
    return 0;
  const int per = p0 < p1 ? p0 : p1;
  return cus * (per > 0 ? per : 0);
}

}  // namespace rheed
