// Angular-spectrum propagation of recorded fields on gfx950: the second
// stage of the two-stage scheme (Sec. 4.4), which carries the field traced
// onto a wave recording plane to the hologram plane; the angular spectrum is
// the field's Fourier transform (Sec. 3).
//
// Per field [h][w] (complex64), zero-padded to [Py][Px] (powers of two,
// >= 2h, >= 2w), with the field in the top-left corner:
//   k_fft_rows     FFT of the h non-zero rows, length Px       [h][w]  -> A [h][Px]
//   k_transpose    A -> B [Px][h]
//   k_fft_columns  per column: zero-pad to Py, FFT, multiply by the transfer
//                  function, inverse FFT, keep rows [0, h)     B -> B
//   k_transpose    B -> A [h][Px]
//   k_ifft_rows    inverse FFT of each row, keep [0, w), scale 1/(Px Py)
// Transfer function H = exp(+i 2 pi z sqrt(1/lambda^2 - f^2)) on propagating
// frequencies (phase reduced in FP64), optionally band-limited
// (Matsushima and Shimobaba, 2009) and cut by a circular pupil, 0 on
// evanescent ones.
//
// Focal stacks (reconstruction): the row spectra of a set of fields (the
// first two steps) are kept and reused for every observation plane; per
// plane the column pass writes to a second buffer and k_ifft_rows_intensity
// sums |u|^2 over the fields instead of writing the fields.
//
// Line FFTs run in LDS, one workgroup per line: Stockham stages
// (Govindaraju et al., SC 2008 formulation) of radix 16 while they fit, then
// radix 4, then a radix-2 stage for an odd remainder; each stage reads its
// operands into registers, synchronises, and writes the results back in
// place. Twiddles come from a table of
// exp(-2 pi i m / n), m < n, per transform length, built once per call in FP64.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "asm.hpp"

namespace hpt {
namespace {

constexpr int kFftThreads = 256;
constexpr int kFftMax = 8192;   // longest line (LDS: 64 KB of complex64)

struct C2 { float x, y; };

// LDS index of element i of a line of up to 4 * U4 * kFftThreads values:
// one pad slot after every 16 elements, so that the strided writes of the
// early Stockham stages (4 and 16 elements apart) spread over the banks.
// Lines of 8192 values (U4 = 8) are not padded: they fill 64 KB of LDS.
template <int U4>
__device__ __forceinline__ uint32_t pd(uint32_t i) { return U4 < 8 ? i + (i >> 4) : i; }
template <int U4>
constexpr size_t lds_bytes(uint32_t n) { return (U4 < 8 ? n + n / 16 : n) * sizeof(C2); }
__device__ __forceinline__ C2 c2(float x, float y) { return {x, y}; }
__device__ __forceinline__ C2 add(C2 a, C2 b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ C2 sub(C2 a, C2 b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ C2 mul(C2 a, C2 b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
// multiply by -i (forward) or +i (inverse)
__device__ __forceinline__ C2 rot(C2 a, bool inv) { return inv ? c2(-a.y, a.x) : c2(a.y, -a.x); }

// exp(s 2 pi i m / n) with s = -1 forward, +1 inverse, from the table
// tw[m] = exp(-2 pi i m / n) of the transform length n.
__device__ __forceinline__ C2 twiddle(const float2 *tw, uint32_t m, bool inv) {
  const float2 v = tw[m];
  return c2(v.x, inv ? -v.y : v.y);
}

// Radix-4 DFT of a[0..3] in place (forward: exp(-2 pi i), inverse: +).
__device__ __forceinline__ void dft4(C2 &a0, C2 &a1, C2 &a2, C2 &a3, bool inv) {
  C2 b0 = add(a0, a2), b1 = sub(a0, a2), b2 = add(a1, a3), b3 = rot(sub(a1, a3), inv);
  a0 = add(b0, b2);
  a1 = add(b1, b3);
  a2 = sub(b0, b2);
  a3 = sub(b1, b3);
}

// Radix-16 DFT of a[0..15] in place, as 4 x 4: DFT-4 over n1 of a[4 n1 + n2]
// for each n2, twiddles exp(-+2 pi i n2 k1 / 16), DFT-4 over n2; output k =
// k1 + 4 k2 lands in a[k].
__device__ __forceinline__ void dft16(C2 (&a)[16], bool inv) {
  // exp(-2 pi i m / 16), m = 0..9
  constexpr float c1 = 0.923879532511286756f, s1 = 0.382683432365089772f, h = 0.707106781186547524f;
  const float cs[10][2] = {{1.f, 0.f}, {c1, -s1}, {h, -h}, {s1, -c1}, {0.f, -1.f},
                           {-s1, -c1}, {-h, -h}, {-c1, -s1}, {-1.f, 0.f}, {-c1, s1}};
  C2 t[16];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    C2 b0 = a[n2], b1 = a[n2 + 4], b2 = a[n2 + 8], b3 = a[n2 + 12];
    dft4(b0, b1, b2, b3, inv);
    t[4 * n2 + 0] = b0; t[4 * n2 + 1] = b1; t[4 * n2 + 2] = b2; t[4 * n2 + 3] = b3;   // t[n2][k1]
  }
#pragma unroll
  for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1) {
      const int m = n2 * k1;
      t[4 * n2 + k1] = mul(t[4 * n2 + k1], c2(cs[m][0], inv ? -cs[m][1] : cs[m][1]));
    }
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    C2 b0 = t[k1], b1 = t[4 + k1], b2 = t[8 + k1], b3 = t[12 + k1];
    dft4(b0, b1, b2, b3, inv);
    a[k1] = b0; a[k1 + 4] = b1; a[k1 + 8] = b2; a[k1 + 12] = b3;
  }
}

// One Stockham radix-16 stage of an n-point FFT in LDS (all threads take
// part; reads, synchronises, writes, synchronises): butterfly j takes
// x[j + r n/16], r < 16, twiddled by exp(-+2 pi i r k / (16 Ns)), k = j mod
// Ns, and writes its 16-point DFT to x[(j / Ns) 16 Ns + k + r Ns].
template <int U4>
__device__ __forceinline__ void stage16(C2 *x, uint32_t n, uint32_t Ns, bool inv, const float2 *tw) {
  constexpr int U16 = (U4 + 3) / 4;
  const uint32_t tid = threadIdx.x;
  const uint32_t q16 = n / 16;
  {
    C2 v[U16][16];
#pragma unroll
    for (int u = 0; u < U16; ++u) {
      const uint32_t j = tid + (uint32_t)u * kFftThreads;
      if (j < q16) {
        const uint32_t k = j % Ns;
#pragma unroll
        for (int r = 0; r < 16; ++r) v[u][r] = x[pd<U4>(j + (uint32_t)r * q16)];
        if (Ns > 1) {  // exp(-+2 pi i r k / (16 Ns)) = tw[r k n / (16 Ns)]
          const uint32_t st = k * (n / (16 * Ns));
#pragma unroll
          for (int r = 1; r < 16; ++r) v[u][r] = mul(v[u][r], twiddle(tw, (uint32_t)r * st, inv));
        }
        dft16(v[u], inv);
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U16; ++u) {
      const uint32_t j = tid + (uint32_t)u * kFftThreads;
      if (j < q16) {
        const uint32_t d = (j / Ns) * Ns * 16 + j % Ns;
#pragma unroll
        for (int r = 0; r < 16; ++r) x[pd<U4>(d + (uint32_t)r * Ns)] = v[u][r];
      }
    }
    __syncthreads();
  }
}

// In-place FFT of the n = 2^lg values in LDS buffer x (all threads of the
// block take part; returns synchronised): Stockham radix-16 stages while
// they fit, then radix-4, then a radix-2 stage for odd remainders. Each
// thread handles butterflies j = tid + u * kFftThreads; the per-thread
// operands stay in registers (static indices), written back after the whole
// stage has been read. U4: n <= 4 * U4 * kFftThreads.
template <int U4>
__device__ void lds_fft(C2 *x, uint32_t n, uint32_t lg, bool inv, const float2 *tw) {
  constexpr int U2 = 2 * U4;
  const uint32_t tid = threadIdx.x;
  uint32_t Ns = 1;
  for (uint32_t s = 0; s < lg / 4; ++s) {
    stage16<U4>(x, n, Ns, inv, tw);
    Ns *= 16;
  }
  const uint32_t q = n / 4;
  for (uint32_t s = 0; s < (lg % 4) / 2; ++s) {
    C2 v[U4][4];
#pragma unroll
    for (int u = 0; u < U4; ++u) {
      const uint32_t j = tid + (uint32_t)u * kFftThreads;
      if (j < q) {
        const uint32_t k = j % Ns;
        C2 a0 = x[pd<U4>(j)], a1 = x[pd<U4>(j + q)], a2 = x[pd<U4>(j + 2 * q)], a3 = x[pd<U4>(j + 3 * q)];
        if (Ns > 1) {  // exp(-+2 pi i e k / (4 Ns)) = tw[e k n / (4 Ns)]
          const uint32_t st = k * (n / (4 * Ns));
          a1 = mul(a1, twiddle(tw, st, inv));
          a2 = mul(a2, twiddle(tw, 2 * st, inv));
          a3 = mul(a3, twiddle(tw, 3 * st, inv));
        }
        C2 b0 = add(a0, a2), b1 = sub(a0, a2), b2 = add(a1, a3), b3 = rot(sub(a1, a3), inv);
        v[u][0] = add(b0, b2);
        v[u][1] = add(b1, b3);
        v[u][2] = sub(b0, b2);
        v[u][3] = sub(b1, b3);
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U4; ++u) {
      const uint32_t j = tid + (uint32_t)u * kFftThreads;
      if (j < q) {
        const uint32_t d = (j / Ns) * Ns * 4 + j % Ns;
        x[pd<U4>(d)] = v[u][0];
        x[pd<U4>(d + Ns)] = v[u][1];
        x[pd<U4>(d + 2 * Ns)] = v[u][2];
        x[pd<U4>(d + 3 * Ns)] = v[u][3];
      }
    }
    __syncthreads();
    Ns *= 4;
  }
  if (lg & 1u) {  // final radix-2 stage
    const uint32_t hn = n / 2;
    C2 v[U2][2];
#pragma unroll
    for (int u = 0; u < U2; ++u) {
      const uint32_t j = tid + (uint32_t)u * kFftThreads;
      if (j < hn) {
        C2 a0 = x[pd<U4>(j)], a1 = x[pd<U4>(j + hn)];
        if (Ns > 1) a1 = mul(a1, twiddle(tw, (j % Ns) * (n / (2 * Ns)), inv));
        v[u][0] = add(a0, a1);
        v[u][1] = sub(a0, a1);
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U2; ++u) {
      const uint32_t j = tid + (uint32_t)u * kFftThreads;
      if (j < hn) {
        const uint32_t d = (j / Ns) * Ns * 2 + j % Ns;
        x[pd<U4>(d)] = v[u][0];
        x[pd<U4>(d + Ns)] = v[u][1];
      }
    }
    __syncthreads();
  }
}

// Forward FFT of row (f, y) of in [nf][h][w], zero-padded to Px -> A [nf][h][Px].
template <int U4>
__global__ void __launch_bounds__(kFftThreads) k_fft_rows(const float2 *in, float2 *A, uint32_t w, uint32_t h,
                                                          uint32_t px, uint32_t lgx, const float2 *tw) {
  extern __shared__ C2 lds[];
  const size_t row = blockIdx.x;  // f * h + y
  const float2 *src = in + row * w;
  for (uint32_t i = threadIdx.x; i < px; i += kFftThreads) {
    float2 v = i < w ? src[i] : make_float2(0.f, 0.f);
    lds[pd<U4>(i)] = c2(v.x, v.y);
  }
  __syncthreads();
  lds_fft<U4>(lds, px, lgx, false, tw);
  float2 *dst = A + row * px;
  for (uint32_t i = threadIdx.x; i < px; i += kFftThreads) dst[i] = make_float2(lds[pd<U4>(i)].x, lds[pd<U4>(i)].y);
}

// Transpose of each of nf matrices [rows][cols] -> [cols][rows], 32 x 32 tiles.
__global__ void __launch_bounds__(256) k_transpose(const float2 *in, float2 *out, uint32_t rows, uint32_t cols) {
  __shared__ float2 tile[32][33];
  const uint32_t f = blockIdx.z;
  const uint32_t c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const float2 *src = in + (size_t)f * rows * cols;
  float2 *dst = out + (size_t)f * rows * cols;
  const uint32_t tx = threadIdx.x & 31u, ty = threadIdx.x >> 5;  // 32 x 8
  for (uint32_t k = ty; k < 32; k += 8) {
    uint32_t r = r0 + k, c = c0 + tx;
    if (r < rows && c < cols) tile[k][tx] = src[(size_t)r * cols + c];
  }
  __syncthreads();
  for (uint32_t k = ty; k < 32; k += 8) {
    uint32_t c = c0 + k, r = r0 + tx;
    if (r < rows && c < cols) dst[(size_t)c * rows + r] = tile[tx][k];
  }
}

// Column kx of all nf fields: B [nf][Px][h] holds the row spectra
// transposed. The transfer function of the column is computed once (each
// thread keeps its rows' values in registers) and applied to every field:
// zero-pad the column to Py, FFT, multiply by H(f_x, f_y), inverse FFT, keep
// rows [0, h).
template <int U4>
__global__ void __launch_bounds__(kFftThreads) k_fft_columns(const float2 *src, float2 *dst, uint32_t nf,
                                                             uint32_t h, uint32_t px, uint32_t py, uint32_t lgy,
                                                             AsmParams P, const float2 *tw) {
  extern __shared__ C2 lds[];
  constexpr int UH = 4 * U4;  // rows per thread (py <= 4 * U4 * kFftThreads)
  const uint32_t kx = blockIdx.x, t = threadIdx.x;
  // FFT frequency order: k / (P d) for k < P/2, (k - P) / (P d) otherwise
  const double fx = (kx < px / 2 ? (double)kx : (double)kx - (double)px) * P.dfx;
  const bool ok_x = !P.band_limit || fabs(fx) <= P.lim_x;
  C2 Hr[UH];
#pragma unroll
  for (int u = 0; u < UH; ++u) {
    const uint32_t i = t + (uint32_t)u * kFftThreads;
    Hr[u] = c2(0.f, 0.f);
    if (i < py) {
      const double fy = (i < py / 2 ? (double)i : (double)i - (double)py) * P.dfy;
      const double f2 = fx * fx + fy * fy;
      if (ok_x && (!P.band_limit || fabs(fy) <= P.lim_y) && f2 < P.inv_lam2 &&
          (P.pupil2 <= 0.0 || f2 <= P.pupil2)) {
        // z sqrt(1/lambda^2 - f^2) = z/lambda - z f^2 / (1/lambda + sqrt(1/lambda^2 - f^2)),
        // the first term reduced modulo 1 on the host
        const double rev = P.z_rev_frac - P.z * f2 / (P.inv_lam + sqrt(P.inv_lam2 - f2));
        const double fr = rev - floor(rev);
        double sn, cs;
        sincospi(2.0 * fr, &sn, &cs);
        Hr[u] = c2((float)cs, (float)sn);
      }
    }
  }
  if constexpr (U4 == 4) {
    // 4096-point columns: the three radix-16 stages of each transform map
    // thread t to elements t + 256 r at both ends, so the first forward stage
    // reads the column from global memory, the last forward stage, the
    // transfer function and the first inverse stage stay in registers, and
    // the last inverse stage writes rows [0, h) to global memory: 4 LDS
    // passes per field instead of 8 plus the multiply pass.
    for (uint32_t f = 0; f < nf; ++f) {
      const float2 *scol = src + ((size_t)f * px + kx) * h;
      float2 *col = dst + ((size_t)f * px + kx) * h;
      C2 v[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const uint32_t i = t + (uint32_t)r * kFftThreads;
        const float2 g = i < h ? scol[i] : make_float2(0.f, 0.f);
        v[r] = c2(g.x, g.y);
      }
      dft16(v, false);                                   // forward stage, Ns = 1
      __syncthreads();                                   // the previous field's last reads are done
#pragma unroll
      for (int r = 0; r < 16; ++r) lds[pd<U4>(16 * t + (uint32_t)r)] = v[r];
      __syncthreads();
      stage16<U4>(lds, py, 16, false, tw);               // forward stage, Ns = 16
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = lds[pd<U4>(t + (uint32_t)r * kFftThreads)];
#pragma unroll
      for (int r = 1; r < 16; ++r) v[r] = mul(v[r], twiddle(tw, (uint32_t)r * t, false));
      dft16(v, false);                                   // forward stage, Ns = 256: v[r] = X[t + 256 r]
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = mul(v[r], Hr[r]);
      dft16(v, true);                                    // inverse stage, Ns = 1
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 16; ++r) lds[pd<U4>(16 * t + (uint32_t)r)] = v[r];
      __syncthreads();
      stage16<U4>(lds, py, 16, true, tw);                // inverse stage, Ns = 16
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = lds[pd<U4>(t + (uint32_t)r * kFftThreads)];
#pragma unroll
      for (int r = 1; r < 16; ++r) v[r] = mul(v[r], twiddle(tw, (uint32_t)r * t, true));
      dft16(v, true);                                    // inverse stage, Ns = 256
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const uint32_t i = t + (uint32_t)r * kFftThreads;
        if (i < h) col[i] = make_float2(v[r].x, v[r].y);
      }
    }
    return;
  }
  for (uint32_t f = 0; f < nf; ++f) {
    const float2 *scol = src + ((size_t)f * px + kx) * h;
    float2 *col = dst + ((size_t)f * px + kx) * h;
    for (uint32_t i = t; i < py; i += kFftThreads) {
      float2 v = i < h ? scol[i] : make_float2(0.f, 0.f);
      lds[pd<U4>(i)] = c2(v.x, v.y);
    }
    __syncthreads();
    lds_fft<U4>(lds, py, lgy, false, tw);
#pragma unroll
    for (int u = 0; u < UH; ++u) {
      const uint32_t i = t + (uint32_t)u * kFftThreads;
      if (i < py) lds[pd<U4>(i)] = mul(lds[pd<U4>(i)], Hr[u]);
    }
    __syncthreads();
    lds_fft<U4>(lds, py, lgy, true, tw);
    for (uint32_t i = t; i < h; i += kFftThreads) col[i] = make_float2(lds[pd<U4>(i)].x, lds[pd<U4>(i)].y);
    __syncthreads();  // before the next field overwrites the buffer
  }
}

// tw[m] = exp(-2 pi i m / n), m < n (FP64, rounded).
__global__ void k_twiddles(float2 *tw, uint32_t n) {
  const uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  double sn, cs;
  sincospi(2.0 * (double)m / (double)n, &sn, &cs);
  tw[m] = make_float2((float)cs, (float)-sn);
}

// Inverse FFT of row (f, y) of A [nf][h][Px]; keep [0, w), scale -> out [nf][h][w].
template <int U4>
__global__ void __launch_bounds__(kFftThreads) k_ifft_rows(const float2 *A, float2 *out, uint32_t w, uint32_t h,
                                                           uint32_t px, uint32_t lgx, float scale,
                                                           const float2 *tw) {
  extern __shared__ C2 lds[];
  const size_t row = blockIdx.x;
  const float2 *src = A + row * px;
  for (uint32_t i = threadIdx.x; i < px; i += kFftThreads) {
    float2 v = src[i];
    lds[pd<U4>(i)] = c2(v.x, v.y);
  }
  __syncthreads();
  lds_fft<U4>(lds, px, lgx, true, tw);
  float2 *dst = out + row * w;
  for (uint32_t i = threadIdx.x; i < w; i += kFftThreads) dst[i] = make_float2(lds[pd<U4>(i)].x * scale, lds[pd<U4>(i)].y * scale);
}

// Summed intensity of row y over nf fields: inverse FFT of row (f, y) of
// A [nf][h][Px] for every f < nf, scaled by 1/(Px Py), |.|^2 of the first w
// values summed over f, times `weight`; written into (or added to) I [h][w].
template <int U4>
__global__ void __launch_bounds__(kFftThreads) k_ifft_rows_intensity(const float2 *A, float *I, uint32_t nf,
                                                                     uint32_t w, uint32_t h, uint32_t px,
                                                                     uint32_t lgx, float scale, float weight,
                                                                     uint32_t accumulate, const float2 *tw) {
  extern __shared__ C2 lds[];
  constexpr int UW = 4 * U4;  // values per thread (px <= 4 * U4 * kFftThreads)
  const uint32_t y = blockIdx.x, t = threadIdx.x;
  float acc[UW];
#pragma unroll
  for (int u = 0; u < UW; ++u) acc[u] = 0.f;
  for (uint32_t f = 0; f < nf; ++f) {
    const float2 *src = A + ((size_t)f * h + y) * px;
    for (uint32_t i = t; i < px; i += kFftThreads) {
      float2 v = src[i];
      lds[pd<U4>(i)] = c2(v.x, v.y);
    }
    __syncthreads();
    lds_fft<U4>(lds, px, lgx, true, tw);
#pragma unroll
    for (int u = 0; u < UW; ++u) {
      const uint32_t i = t + (uint32_t)u * kFftThreads;
      if (i < w) {
        const float re = lds[pd<U4>(i)].x * scale, im = lds[pd<U4>(i)].y * scale;
        acc[u] += re * re + im * im;
      }
    }
    __syncthreads();  // before the next field overwrites the buffer
  }
  float *dst = I + (size_t)y * w;
#pragma unroll
  for (int u = 0; u < UW; ++u) {
    const uint32_t i = t + (uint32_t)u * kFftThreads;
    if (i < w) dst[i] = (accumulate ? dst[i] : 0.f) + acc[u] * weight;
  }
}

uint32_t log2u(uint32_t n) {
  uint32_t l = 0;
  while ((1u << l) < n) ++l;
  return l;
}

template <int U4>
void launch_rows(bool inv, const float2 *in, float2 *out, uint32_t nrows, uint32_t w, uint32_t h, uint32_t px,
                 uint32_t lgx, float scale, const float2 *tw, hipStream_t st) {
  if (!inv)
    hipLaunchKernelGGL(k_fft_rows<U4>, dim3(nrows), dim3(kFftThreads), lds_bytes<U4>(px), st, in, out, w, h, px, lgx,
                       tw);
  else
    hipLaunchKernelGGL(k_ifft_rows<U4>, dim3(nrows), dim3(kFftThreads), lds_bytes<U4>(px), st, in, out, w, h, px, lgx,
                       scale, tw);
}

void rows(bool inv, const float2 *in, float2 *out, uint32_t nrows, uint32_t w, uint32_t h, uint32_t px,
          uint32_t lgx, float scale, const float2 *tw, hipStream_t st) {
  if (px <= 4 * kFftThreads) launch_rows<1>(inv, in, out, nrows, w, h, px, lgx, scale, tw, st);
  else if (px <= 8 * kFftThreads) launch_rows<2>(inv, in, out, nrows, w, h, px, lgx, scale, tw, st);
  else if (px <= 16 * kFftThreads) launch_rows<4>(inv, in, out, nrows, w, h, px, lgx, scale, tw, st);
  else launch_rows<8>(inv, in, out, nrows, w, h, px, lgx, scale, tw, st);
}

void columns(const float2 *src, float2 *dst, uint32_t nf, uint32_t h, uint32_t px, uint32_t py, uint32_t lgy,
             const AsmParams &P, const float2 *tw, hipStream_t st) {
  if (py <= 4 * kFftThreads)
    hipLaunchKernelGGL(k_fft_columns<1>, dim3(px), dim3(kFftThreads), lds_bytes<1>(py), st, src, dst, nf, h, px, py,
                       lgy, P, tw);
  else if (py <= 8 * kFftThreads)
    hipLaunchKernelGGL(k_fft_columns<2>, dim3(px), dim3(kFftThreads), lds_bytes<2>(py), st, src, dst, nf, h, px, py,
                       lgy, P, tw);
  else if (py <= 16 * kFftThreads)
    hipLaunchKernelGGL(k_fft_columns<4>, dim3(px), dim3(kFftThreads), lds_bytes<4>(py), st, src, dst, nf, h, px, py,
                       lgy, P, tw);
  else
    hipLaunchKernelGGL(k_fft_columns<8>, dim3(px), dim3(kFftThreads), lds_bytes<8>(py), st, src, dst, nf, h, px, py,
                       lgy, P, tw);
}

template <int U4>
void launch_intensity_rows(const float2 *A, float *I, uint32_t nf, uint32_t w, uint32_t h, uint32_t px,
                           uint32_t lgx, float scale, float weight, bool accumulate, const float2 *tw,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_ifft_rows_intensity<U4>, dim3(h), dim3(kFftThreads), lds_bytes<U4>(px), st, A, I, nf, w, h, px,
                     lgx, scale, weight, accumulate ? 1u : 0u, tw);
}

void intensity_rows(const float2 *A, float *I, uint32_t nf, uint32_t w, uint32_t h, uint32_t px, uint32_t lgx,
                    float scale, float weight, bool accumulate, const float2 *tw, hipStream_t st) {
  if (px <= 4 * kFftThreads) launch_intensity_rows<1>(A, I, nf, w, h, px, lgx, scale, weight, accumulate, tw, st);
  else if (px <= 8 * kFftThreads) launch_intensity_rows<2>(A, I, nf, w, h, px, lgx, scale, weight, accumulate, tw, st);
  else if (px <= 16 * kFftThreads) launch_intensity_rows<4>(A, I, nf, w, h, px, lgx, scale, weight, accumulate, tw, st);
  else launch_intensity_rows<8>(A, I, nf, w, h, px, lgx, scale, weight, accumulate, tw, st);
}

}  // namespace

// Scratch of the allocation-free propagation (hpt_asm_propagate_noalloc):
// one array per device, held until the process ends. Host code never names
// it directly (its host-side name is a stand-in, not a device address): the
// device address comes from asm_noalloc_scratch().
static __device__ __align__(256) float2 scratch[kNoAllocScratchElems];

hipError_t asm_noalloc_scratch(int device, float2 **ptr) {
  static std::mutex mu;
  static std::map<int, float2 *> table;
  std::lock_guard<std::mutex> g(mu);
  auto it = table.find(device);
  if (it != table.end()) { *ptr = it->second; return hipSuccess; }
  float2 *p = nullptr;
  hipError_t e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  table[device] = p;
  *ptr = p;
  return hipSuccess;
}

uint32_t asm_padded(uint32_t n) {
  uint32_t p = 1;
  while (p < 2 * n) p *= 2;
  return p;
}

hipError_t launch_asm_twiddles(float2 *tw, uint32_t w, uint32_t h, hipStream_t st) {
  const uint32_t px = asm_padded(w), py = asm_padded(h);
  hipLaunchKernelGGL(k_twiddles, dim3((px + 255) / 256), dim3(256), 0, st, tw, px);
  hipLaunchKernelGGL(k_twiddles, dim3((py + 255) / 256), dim3(256), 0, st, tw + px, py);
  return hipGetLastError();
}

hipError_t launch_asm_spectra(const float2 *in, float2 *A, float2 *B0, const float2 *tw, uint32_t nf, uint32_t w,
                              uint32_t h, hipStream_t st) {
  const uint32_t px = asm_padded(w), py = asm_padded(h);
  if (px > (uint32_t)kFftMax || py > (uint32_t)kFftMax || nf == 0 || w == 0 || h == 0) return hipErrorInvalidValue;
  rows(false, in, A, nf * h, w, h, px, log2u(px), 1.0f, tw, st);
  hipLaunchKernelGGL(k_transpose, dim3((px + 31) / 32, (h + 31) / 32, nf), dim3(256), 0, st, A, B0, h, px);
  return hipGetLastError();
}

hipError_t launch_asm_intensity(const float2 *B0, float2 *B, float2 *A, const float2 *tw, uint32_t nf, uint32_t w,
                                uint32_t h, const AsmParams &P, float *I, float weight, bool accumulate,
                                hipStream_t st) {
  const uint32_t px = asm_padded(w), py = asm_padded(h);
  if (px > (uint32_t)kFftMax || py > (uint32_t)kFftMax || nf == 0 || w == 0 || h == 0) return hipErrorInvalidValue;
  columns(B0, B, nf, h, px, py, log2u(py), P, tw + px, st);
  hipLaunchKernelGGL(k_transpose, dim3((h + 31) / 32, (px + 31) / 32, nf), dim3(256), 0, st, B, A, px, h);
  intensity_rows(A, I, nf, w, h, px, log2u(px), 1.0f / ((float)px * (float)py), weight, accumulate, tw, st);
  return hipGetLastError();
}

hipError_t launch_asm(const float2 *in, float2 *out, float2 *A, float2 *B, const float2 *tw, uint32_t nf,
                      uint32_t w, uint32_t h, const AsmParams &P, hipStream_t st) {
  const uint32_t px = asm_padded(w), py = asm_padded(h);
  if (px > (uint32_t)kFftMax || py > (uint32_t)kFftMax || nf == 0 || w == 0 || h == 0) return hipErrorInvalidValue;
  const uint32_t lgx = log2u(px), lgy = log2u(py);
  rows(false, in, A, nf * h, w, h, px, lgx, 1.0f, tw, st);
  hipLaunchKernelGGL(k_transpose, dim3((px + 31) / 32, (h + 31) / 32, nf), dim3(256), 0, st, A, B, h, px);
  columns(B, B, nf, h, px, py, lgy, P, tw + px, st);
  hipLaunchKernelGGL(k_transpose, dim3((h + 31) / 32, (px + 31) / 32, nf), dim3(256), 0, st, B, A, px, h);
  rows(true, A, out, nf * h, w, h, px, lgx, 1.0f / ((float)px * (float)py), tw, st);
  return hipGetLastError();
}

}  // namespace hpt
