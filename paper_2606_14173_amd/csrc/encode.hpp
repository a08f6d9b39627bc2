// Phase-only encoding launchers (Adam under complex-amplitude supervision).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace hpt {

// Adam constants (Kingma and Ba, 2015).
constexpr float kAdamBeta1 = 0.9f, kAdamBeta2 = 0.999f, kAdamEps = 1e-8f;

// Blocks per field of the dot-product pass (the partial-sum buffer holds
// nf * enc_dot_blocks(hw) * 3 doubles).
uint32_t enc_dot_blocks(uint32_t hw);

// phi = arg U (0 where U = 0) unless warm (phi kept); a = exp(i phi). n values.
hipError_t launch_enc_init(const float2 *U, float *phi, float2 *a, size_t n, bool warm, hipStream_t st);
// vv[f] = <V_f, V_f> for nf fields of hw values.
hipError_t launch_enc_norm(const float2 *V, double *part, double *vv, uint32_t nf, uint32_t hw, hipStream_t st);
// s[f] = <V_f, A_f> / vv[f]; rel[f] = 1 - |<V_f, A_f>|^2 / (vv[f] <A_f, A_f>).
hipError_t launch_enc_scale(const float2 *A, const float2 *V, double *part, const double *vv, double2 *s,
                            double *rel, uint32_t nf, uint32_t hw, hipStream_t st);
// A_f -= s[f] V_f.
hipError_t launch_enc_residual(float2 *A, const float2 *V, const double2 *s, uint32_t nf, uint32_t hw,
                               hipStream_t st);
// g = 2 Im(G conj(a)); Adam step with bias corrections bc1 = 1 - beta1^k,
// bc2 = 1 - beta2^k; a = exp(i phi) of the new phase. n values.
hipError_t launch_enc_adam(float *phi, float *m, float *v, float2 *a, const float2 *G, size_t n, float lr,
                           float bc1, float bc2, hipStream_t st);

}  // namespace hpt
