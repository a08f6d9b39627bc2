// Phase-only encoding on gfx950: Adam on the SLM phase under complex-amplitude
// supervision on one plane with a phase-shift-invariant scale factor (the
// paper's hologram encoding, Sec. 2 and Sec. 5.3). Per field and step:
//   A = P_z exp(i phi)                          (ASM, asm.hip)
//   s = <V, A> / <V, V>, L = ||A - s V||^2      k_enc_dots + k_enc_scale
//   R = A - s V                                 k_enc_residual
//   G = P_{-z} R                                (ASM: the adjoint of P_z)
//   g = 2 Im(G conj(a)); Adam; a = exp(i phi)   k_enc_adam
// Fields are [n][h][w] complex64; phases and Adam moments [n][h][w] float32;
// the dot products accumulate in FP64 in a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include "encode.hpp"

namespace hpt {
namespace {

constexpr int kEncBlock = 256;

__global__ void __launch_bounds__(kEncBlock) k_enc_init(const float2 *U, float *phi, float2 *a, size_t n,
                                                        uint32_t warm) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float p;
  if (warm) {
    p = phi[i];
  } else {
    const float2 u = U[i];
    p = (u.x == 0.f && u.y == 0.f) ? 0.f : atan2f(u.y, u.x);
    phi[i] = p;
  }
  float sn, cs;
  sincosf(p, &sn, &cs);
  a[i] = make_float2(cs, sn);
}

// Partial sums over block x of field f = blockIdx.y: sum conj(V) A (re, im)
// and sum |A|^2, in FP64 -> part[(f * gridDim.x + x) * 3 + k].
__global__ void __launch_bounds__(kEncBlock) k_enc_dots(const float2 *A, const float2 *V, double *part,
                                                        uint32_t hw) {
  __shared__ double sh[3][kEncBlock];
  const uint32_t f = blockIdx.y, t = threadIdx.x;
  const float2 *Af = A + (size_t)f * hw, *Vf = V + (size_t)f * hw;
  double dr = 0.0, di = 0.0, aa = 0.0;
  for (uint32_t i = blockIdx.x * kEncBlock + t; i < hw; i += gridDim.x * kEncBlock) {
    const float2 x = Af[i], v = Vf[i];
    dr += (double)v.x * x.x + (double)v.y * x.y;
    di += (double)v.x * x.y - (double)v.y * x.x;
    aa += (double)x.x * x.x + (double)x.y * x.y;
  }
  sh[0][t] = dr; sh[1][t] = di; sh[2][t] = aa;
  __syncthreads();
  for (uint32_t s = kEncBlock / 2; s > 0; s >>= 1) {
    if (t < s)
      for (int k = 0; k < 3; ++k) sh[k][t] += sh[k][t + s];
    __syncthreads();
  }
  if (t < 3) part[((size_t)f * gridDim.x + blockIdx.x) * 3 + t] = sh[t][0];
}

// Per field: the optimal scale s = <V, A> / <V, V> and the relative loss
// 1 - |<V, A>|^2 / (<V, V> <A, A>); vv[f] = <V, V>.
__global__ void k_enc_scale(const double *part, uint32_t nb, uint32_t n, const double *vv, double2 *s,
                            double *rel) {
  const uint32_t f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n) return;
  double dr = 0.0, di = 0.0, aa = 0.0;
  for (uint32_t b = 0; b < nb; ++b) {
    const double *p = part + ((size_t)f * nb + b) * 3;
    dr += p[0]; di += p[1]; aa += p[2];
  }
  const double v = vv[f];
  s[f] = v > 0.0 ? make_double2(dr / v, di / v) : make_double2(0.0, 0.0);
  rel[f] = (v > 0.0 && aa > 0.0) ? 1.0 - (dr * dr + di * di) / (v * aa) : 1.0;
}

// <V, V> per field from the third partial of k_enc_dots(V, V).
__global__ void k_enc_norm(const double *part, uint32_t nb, uint32_t n, double *vv) {
  const uint32_t f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n) return;
  double aa = 0.0;
  for (uint32_t b = 0; b < nb; ++b) aa += part[((size_t)f * nb + b) * 3 + 2];
  vv[f] = aa;
}

__global__ void __launch_bounds__(kEncBlock) k_enc_residual(float2 *A, const float2 *V, const double2 *s,
                                                            uint32_t hw, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 sf = s[i / hw];
  const float sr = (float)sf.x, si = (float)sf.y;
  const float2 v = V[i], x = A[i];
  A[i] = make_float2(x.x - (sr * v.x - si * v.y), x.y - (sr * v.y + si * v.x));
}

__global__ void __launch_bounds__(kEncBlock) k_enc_adam(float *phi, float *m, float *v, float2 *a,
                                                        const float2 *G, size_t n, float lr, float bc1,
                                                        float bc2) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float2 g2 = G[i], ai = a[i];
  const float g = 2.0f * (g2.y * ai.x - g2.x * ai.y);  // 2 Im(G conj(a))
  const float mi = kAdamBeta1 * m[i] + (1.0f - kAdamBeta1) * g;
  const float vi = kAdamBeta2 * v[i] + (1.0f - kAdamBeta2) * g * g;
  m[i] = mi;
  v[i] = vi;
  const float p = phi[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + kAdamEps);
  phi[i] = p;
  float sn, cs;
  sincosf(p, &sn, &cs);
  a[i] = make_float2(cs, sn);
}

inline uint32_t grid1(size_t n) { return (uint32_t)((n + kEncBlock - 1) / kEncBlock); }

}  // namespace

uint32_t enc_dot_blocks(uint32_t hw) {
  const uint32_t b = (hw + kEncBlock * 8 - 1) / (kEncBlock * 8);
  return b < 1 ? 1 : (b > 256 ? 256 : b);
}

hipError_t launch_enc_init(const float2 *U, float *phi, float2 *a, size_t n, bool warm, hipStream_t st) {
  hipLaunchKernelGGL(k_enc_init, dim3(grid1(n)), dim3(kEncBlock), 0, st, U, phi, a, n, warm ? 1u : 0u);
  return hipGetLastError();
}

hipError_t launch_enc_norm(const float2 *V, double *part, double *vv, uint32_t nf, uint32_t hw, hipStream_t st) {
  const uint32_t nb = enc_dot_blocks(hw);
  hipLaunchKernelGGL(k_enc_dots, dim3(nb, nf), dim3(kEncBlock), 0, st, V, V, part, hw);
  hipLaunchKernelGGL(k_enc_norm, dim3((nf + 63) / 64), dim3(64), 0, st, part, nb, nf, vv);
  return hipGetLastError();
}

hipError_t launch_enc_scale(const float2 *A, const float2 *V, double *part, const double *vv, double2 *s,
                            double *rel, uint32_t nf, uint32_t hw, hipStream_t st) {
  const uint32_t nb = enc_dot_blocks(hw);
  hipLaunchKernelGGL(k_enc_dots, dim3(nb, nf), dim3(kEncBlock), 0, st, A, V, part, hw);
  hipLaunchKernelGGL(k_enc_scale, dim3((nf + 63) / 64), dim3(64), 0, st, part, nb, nf, vv, s, rel);
  return hipGetLastError();
}

hipError_t launch_enc_residual(float2 *A, const float2 *V, const double2 *s, uint32_t nf, uint32_t hw,
                               hipStream_t st) {
  const size_t n = (size_t)nf * hw;
  hipLaunchKernelGGL(k_enc_residual, dim3(grid1(n)), dim3(kEncBlock), 0, st, A, V, s, hw, n);
  return hipGetLastError();
}

hipError_t launch_enc_adam(float *phi, float *m, float *v, float2 *a, const float2 *G, size_t n, float lr,
                           float bc1, float bc2, hipStream_t st) {
  hipLaunchKernelGGL(k_enc_adam, dim3(grid1(n)), dim3(kEncBlock), 0, st, phi, m, v, a, G, n, lr, bc1, bc2);
  return hipGetLastError();
}

}  // namespace hpt
