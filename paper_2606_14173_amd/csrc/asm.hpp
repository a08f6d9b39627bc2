// Angular-spectrum propagation launcher (second stage of the two-stage
// scheme, Sec. 4.4).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace hpt {

// Transfer-function constants of one propagation, computed on the host in FP64.
struct AsmParams {
  double dfx, dfy;        // frequency steps 1 / (Px d), 1 / (Py d)
  double lim_x, lim_y;    // band limits 1 / (lambda sqrt((2 z dfx)^2 + 1)) (and y)
  double inv_lam, inv_lam2;
  double z;
  double z_rev_frac;      // frac(z / lambda)
  double pupil2;          // squared pupil cutoff (NA / lambda)^2; 0: no pupil
  uint32_t band_limit;
};

// Padded length of one axis: the next power of two >= 2 n.
uint32_t asm_padded(uint32_t n);

// Complex64 elements of the static scratch of the allocation-free
// propagation (72 MiB: one 1920 x 1080 field, padded to 4096 columns, with
// its two work buffers and the twiddle tables).
constexpr size_t kNoAllocScratchElems = 9437184;
// Device address of that scratch on `device` (which must be current): taken
// once per device with hipGetSymbolAddress and kept for the process.
hipError_t asm_noalloc_scratch(int device, float2 **ptr);

// Twiddle tables for fields of w x h: tw[0, Px) for the rows, tw[Px, Px + Py)
// for the columns (Px, Py: the padded sizes).
hipError_t launch_asm_twiddles(float2 *tw, uint32_t w, uint32_t h, hipStream_t st);

// nf fields in [nf][h][w] -> out (may alias in); A, B: scratch of
// nf * h * asm_padded(w) complex64 each; tw: the tables above.
// hipErrorInvalidValue if a padded axis exceeds 8192 or a size is zero.
hipError_t launch_asm(const float2 *in, float2 *out, float2 *A, float2 *B, const float2 *tw, uint32_t nf,
                      uint32_t w, uint32_t h, const AsmParams &P, hipStream_t st);

// Focal stacks. Row spectra of nf fields: in [nf][h][w] -> B0 [nf][Px][h]
// (A: scratch of nf * h * Px complex64).
hipError_t launch_asm_spectra(const float2 *in, float2 *A, float2 *B0, const float2 *tw, uint32_t nf, uint32_t w,
                              uint32_t h, hipStream_t st);
// The nf fields whose row spectra B0 holds, carried by the transfer function
// of P: weight * sum over the fields of |u|^2 written into (accumulate:
// added to) I [h][w]. B, A: scratch of nf * h * Px complex64 each; B0 is
// kept.
hipError_t launch_asm_intensity(const float2 *B0, float2 *B, float2 *A, const float2 *tw, uint32_t nf, uint32_t w,
                                uint32_t h, const AsmParams &P, float *I, float weight, bool accumulate,
                                hipStream_t st);

}  // namespace hpt
