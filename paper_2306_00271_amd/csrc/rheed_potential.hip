// Potential tables u_g(z) on the RK nodes and their adjoint, on gfx950.
//
// Sec. 2.1: the potential is expanded over the surface reciprocal lattice and
// Eq. (sch2) couples beams j and k through the coefficient of g_j - g_k.  For
// Gaussian atoms v_a(r) = sum_m a_m exp(-b_m |r - r_a|^2) the in-plane
// transform per cell area A is
//   V_g(z) = (1/A) sum_a exp(-i g.rho_a) sum_m a_m (pi/b_m) exp(-|g|^2/(4 b_m)) exp(-b_m (z - z_a)^2)
// and u_g = kappa s (charge - i alpha) V_g (s rescales the slab average to the
// mean inner potential; the host folds kappa s (charge - i alpha) / A into
// StructDev::pref).  These kernels are HBM/ALU light compared with the
// propagation and are written for clarity: one thread per (node, g) entry.
#include <mutex>

#include "rheed_internal.h"

namespace rheed {

__device__ __forceinline__ double node_z(const StructDev& S, int n, int nps, const double* cset) {
  if (n >= S.n_slices * nps) return 0.0;
  const int i = n / nps;
  const int m = n - i * nps;
  return -S.thickness + (i + cset[m]) * S.h;
}

__global__ __launch_bounds__(256) void potential_kernel(PotArgs a) {
  const StructDev S = a.structs[blockIdx.y];
  const long long total = (long long)S.n_nodes * S.box;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int n = (int)(e / S.box);
  const int b = (int)(e - (long long)n * S.box);
  const int W = 2 * S.kd + 1;
  const int dh = b / W - S.hd, dk = b % W - S.kd;
  const double gx = dh * S.recip[0] + dk * S.recip[2];
  const double gy = dh * S.recip[1] + dk * S.recip[3];
  const double g2 = gx * gx + gy * gy;
  double wgt[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) wgt[m] = S.scat_a[m] * (M_PI / S.scat_b[m]) * exp(-g2 / (4.0 * S.scat_b[m]));
  const double z = node_z(S, n, a.nodes_per_slice, a.cset);
  const double* at = a.atoms + 3 * S.atom_off;
  double re = 0.0, im = 0.0;
  for (int ia = 0; ia < S.n_atoms; ++ia) {
    const double x = at[3 * ia], y = at[3 * ia + 1], za = at[3 * ia + 2];
    const double dz2 = (z - za) * (z - za);
    double f = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) f += wgt[m] * exp(-S.scat_b[m] * dz2);
    double sn, cs;
    sincos(gx * x + gy * y, &sn, &cs);
    re += f * cs;   // exp(-i phi) = cos(phi) - i sin(phi)
    im -= f * sn;
  }
  a.U[S.table_off + e] = make_double2(S.pref_re * re - S.pref_im * im, S.pref_re * im + S.pref_im * re);
}

// dL/dr_a = sum_{n,g} Re(conj(dU) du/dr_a), with
// du/dx_a = -i g_x t, du/dy_a = -i g_y t, du/dz_a = pref e^{-i g.rho} sum_m 2 b_m (z - z_a) w_m e^{-b_m dz^2}
// where t is the atom's term of u.  Workgroup (atom, chunk) sums a contiguous
// chunk of the (node, g) entries and writes one partial per chunk;
// potential_bwd_sum_kernel adds the chunks in order (deterministic).
__global__ __launch_bounds__(256) void potential_bwd_kernel(PotBwdArgs a, int n_struct, const long long* atom_struct) {
  const long long ga = blockIdx.x;              // global atom index
  const int chunk = blockIdx.y;
  const int sidx = (int)atom_struct[ga];
  const StructDev S = a.structs[sidx];
  const double x = a.atoms[3 * ga], y = a.atoms[3 * ga + 1], za = a.atoms[3 * ga + 2];
  const long long total = (long long)S.n_nodes * S.box;
  const long long per = (total + PBWD_CHUNKS - 1) / PBWD_CHUNKS;
  const long long e0 = chunk * per, e1 = min(total, e0 + per);
  const int W = 2 * S.kd + 1;
  double sx = 0.0, sy = 0.0, sz = 0.0;
  for (long long e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int n = (int)(e / S.box);
    const int b = (int)(e - (long long)n * S.box);
    const int dh = b / W - S.hd, dk = b % W - S.kd;
    const double gx = dh * S.recip[0] + dk * S.recip[2];
    const double gy = dh * S.recip[1] + dk * S.recip[3];
    const double g2 = gx * gx + gy * gy;
    const double z = node_z(S, n, a.nodes_per_slice, a.cset);
    const double dz = z - za;
    double f = 0.0, fz = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const double t = S.scat_a[m] * (M_PI / S.scat_b[m]) * exp(-g2 / (4.0 * S.scat_b[m])) * exp(-S.scat_b[m] * dz * dz);
      f += t;
      fz += 2.0 * S.scat_b[m] * dz * t;
    }
    double sn, cs;
    sincos(gx * x + gy * y, &sn, &cs);
    // t_u = pref * f * (cs - i sn);  du/dz = pref * fz * (cs - i sn)
    const double pr = S.pref_re, pi = S.pref_im;
    const double tr = pr * f * cs + pi * f * sn, ti = pi * f * cs - pr * f * sn;
    const double zr = pr * fz * cs + pi * fz * sn, zi = pi * fz * cs - pr * fz * sn;
    const double2 du = a.dU[S.table_off + e];
    // Re(conj(du) * (-i g t)) = g * (du.x * ti - du.y * tr) ... with -i t = (ti, -tr)
    const double lat = du.x * ti - du.y * tr;
    sx += gx * lat;
    sy += gy * lat;
    sz += du.x * zr + du.y * zi;
  }
  __shared__ double red[3][256];
  red[0][threadIdx.x] = sx;
  red[1][threadIdx.x] = sy;
  red[2][threadIdx.x] = sz;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      red[0][threadIdx.x] += red[0][threadIdx.x + off];
      red[1][threadIdx.x] += red[1][threadIdx.x + off];
      red[2][threadIdx.x] += red[2][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x < 3) a.partial[(ga * PBWD_CHUNKS + chunk) * 3 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void potential_bwd_sum_kernel(const double* partial, double* datoms, long long n) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;  // atom * 3 + component
  if (c >= n) return;
  const long long ga = c / 3, comp = c - 3 * ga;
  double acc = 0.0;
  for (int k = 0; k < PBWD_CHUNKS; ++k) acc += partial[(ga * PBWD_CHUNKS + k) * 3 + comp];
  datoms[c] = acc;
}

// R-factor of the specular beam: loss = sum_p (I[p][0] - t[p])^2 and
// dL/dI[p][j] = 2 (I[p][0] - t[p]) for j = 0, 0 otherwise.  One workgroup,
// fixed reduction order.
__global__ __launch_bounds__(256) void rfactor_kernel(int n_pairs, int ld, const double* I, const double* t,
                                                      double* loss, double* dI) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int p = threadIdx.x; p < n_pairs; p += blockDim.x) {
    const double diff = I[(long long)p * ld] - t[p];
    acc += diff * diff;
    if (dI) {
      dI[(long long)p * ld] = 2.0 * diff;
      for (int j = 1; j < ld; ++j) dI[(long long)p * ld + j] = 0.0;
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) *loss = red[0];
}

// Partial sums of the potential adjoint for callers that cannot allocate
// (rheed_potential_backward_noalloc): a fixed array in device memory, one copy
// per GPU, held until the process ends.  Host code must not pass the array's
// name to a kernel (in host code it is a stand-in, not a device address): the
// device address comes from hipGetSymbolAddress, once per device, below.
static __device__ __align__(256) double scratch[(size_t)PBWD_STATIC_ATOMS * PBWD_CHUNKS * 3];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t potential_bwd_scratch(double** out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_potential(const PotArgs& a, long long max_elems, hipStream_t stream) {
  dim3 grid((unsigned)((max_elems + 255) / 256), a.n_struct), block(256);
  hipLaunchKernelGGL(potential_kernel, grid, block, 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_potential_bwd(const PotBwdArgs& a, long long n_atoms_total, int n_struct, const long long* atom_struct,
                                hipStream_t stream) {
  hipLaunchKernelGGL(potential_bwd_kernel, dim3((unsigned)n_atoms_total, PBWD_CHUNKS), dim3(256), 0, stream, a, n_struct,
                     atom_struct);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long n = 3 * n_atoms_total;
  hipLaunchKernelGGL(potential_bwd_sum_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, a.partial,
                     a.datoms, n);
  return hipGetLastError();
}

hipError_t launch_rfactor(int n_pairs, int ld, const double* I, const double* t, double* loss, double* dI,
                          hipStream_t stream) {
  hipLaunchKernelGGL(rfactor_kernel, dim3(1), dim3(256), 0, stream, n_pairs, ld, I, t, loss, dI);
  return hipGetLastError();
}

}  // namespace rheed
