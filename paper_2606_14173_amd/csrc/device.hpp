// Device helpers of the gfx950 wave path tracer: counter-based random
// numbers, FP32 BVH traversal with a watertight triangle test, FP64 hit
// refinement for the coherent prefix, and BSDF lobe sampling.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hpt_types.hpp"

namespace hpt {

// ------------------------------------------------------------------ Philox
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32 -> 64-bit
// multiplies with a Weyl-sequence key schedule.
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
  return {c0, c1, c2, c3};
}

// 24-bit uniforms: exact in float and double.
__device__ __forceinline__ float uf(uint32_t w) { return (float)(w >> 8) * 5.9604644775390625e-08f; }
__device__ __forceinline__ double ud(uint32_t w) { return (double)(w >> 8) * 5.9604644775390625e-08; }

// ------------------------------------------------------------------ signature
__device__ __forceinline__ void sig_add(unsigned long long &h, uint32_t w) {
  h ^= (unsigned long long)w;
  h *= 0x100000001b3ull;
}
constexpr unsigned long long kSigInit = 0xcbf29ce484222325ull;

// ------------------------------------------------------------------ vectors
struct F3 { float x, y, z; };
struct D3 { double x, y, z; };
__device__ __forceinline__ F3 f3(float x, float y, float z) { return {x, y, z}; }
__device__ __forceinline__ F3 operator+(F3 a, F3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ F3 operator-(F3 a, F3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ F3 operator*(float s, F3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ float dot(F3 a, F3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ F3 cross(F3 a, F3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ F3 normalize(F3 a) { return (1.0f / sqrtf(dot(a, a))) * a; }

__device__ __forceinline__ D3 operator+(D3 a, D3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ D3 operator-(D3 a, D3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ D3 operator*(double s, D3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ double dot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ D3 cross(D3 a, D3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ D3 normalize(D3 a) { return (1.0 / sqrt(dot(a, a))) * a; }
__device__ __forceinline__ F3 to_f(D3 a) { return {(float)a.x, (float)a.y, (float)a.z}; }
__device__ __forceinline__ D3 to_d(F3 a) { return {a.x, a.y, a.z}; }

// ------------------------------------------------------------------ traversal
// Closest hit so far: distance and leaf-order index of the primitive (-1:
// none). Equal distances go to the lower global id.
struct Hit { float t; int32_t prim; };

// Read-only scene data addressed as global memory (address space 1), so the
// compiler issues global loads (counted by vmcnt only) rather than flat loads.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef const v4f __attribute__((address_space(1))) *GF4;
__device__ __forceinline__ GF4 as_global(const float4 *p) { return (GF4)(const void *)p; }
__device__ __forceinline__ float4 ld4(GF4 p) {
  v4f v = *p;
  return make_float4(v.x, v.y, v.z, v.w);
}
// The same for a pointer of any type that is known to address global memory
// (a pointer read from a descriptor in LDS would otherwise be taken as flat).
// The host pass, which only parses device code, sees plain pointers.
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using GPtr = T __attribute__((address_space(1))) *;
#else
template <class T>
using GPtr = T *;
#endif
template <class T>
__device__ __forceinline__ GPtr<T> glb(T *p) {
  return (GPtr<T>)(void *)p;
}
template <class T>
__device__ __forceinline__ GPtr<const T> glb(const T *p) {
  return (GPtr<const T>)(const void *)p;
}

// Watertight ray/triangle test (Woop, Benthin, Wald, JCGT 2013) in FP32 with
// per-ray shear constants; returns t in (tmin, tbest] or leaves best alone.
struct RayPre {
  F3 o, d;
  int kx, ky, kz;
  float Sx, Sy, Sz;
  F3 inv;
};

__device__ __forceinline__ float comp(F3 v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : v.z); }

__device__ __forceinline__ RayPre ray_pre(F3 o, F3 d) {
  RayPre r;
  r.o = o; r.d = d;
  float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
  int kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
  int kx = kz == 2 ? 0 : kz + 1;
  int ky = kx == 2 ? 0 : kx + 1;
  if (comp(d, kz) < 0.f) { int t = kx; kx = ky; ky = t; }
  r.kx = kx; r.ky = ky; r.kz = kz;
  float dz = comp(d, kz);
  r.Sx = comp(d, kx) / dz; r.Sy = comp(d, ky) / dz; r.Sz = 1.0f / dz;
  // reciprocal direction for the slab tests; zero components become huge
  r.inv.x = 1.0f / (fabsf(d.x) > 1e-30f ? d.x : copysignf(1e-30f, d.x));
  r.inv.y = 1.0f / (fabsf(d.y) > 1e-30f ? d.y : copysignf(1e-30f, d.y));
  r.inv.z = 1.0f / (fabsf(d.z) > 1e-30f ? d.z : copysignf(1e-30f, d.z));
  return r;
}

__device__ __forceinline__ bool tri_hit(const RayPre &r, F3 v0, F3 v1, F3 v2, float tmin, float tbest,
                                        float &t_out) {
  F3 A = v0 - r.o, B = v1 - r.o, C = v2 - r.o;
  float Az = comp(A, r.kz), Bz = comp(B, r.kz), Cz = comp(C, r.kz);
  float Ax = comp(A, r.kx) - r.Sx * Az, Ay = comp(A, r.ky) - r.Sy * Az;
  float Bx = comp(B, r.kx) - r.Sx * Bz, By = comp(B, r.ky) - r.Sy * Bz;
  float Cx = comp(C, r.kx) - r.Sx * Cz, Cy = comp(C, r.ky) - r.Sy * Cz;
  float U = Cx * By - Cy * Bx;
  float V = Ax * Cy - Ay * Cx;
  float W = Bx * Ay - By * Ax;
  if (U == 0.f || V == 0.f || W == 0.f) {
    double CxBy = (double)Cx * By, CyBx = (double)Cy * Bx;
    U = (float)(CxBy - CyBx);
    double AxCy = (double)Ax * Cy, AyCx = (double)Ay * Cx;
    V = (float)(AxCy - AyCx);
    double BxAy = (double)Bx * Ay, ByAx = (double)By * Ax;
    W = (float)(BxAy - ByAx);
  }
  if ((U < 0.f || V < 0.f || W < 0.f) && (U > 0.f || V > 0.f || W > 0.f)) return false;
  float det = U + V + W;
  if (det == 0.f) return false;
  float T = r.Sz * (U * Az + V * Bz + W * Cz);
  float t = T * __builtin_amdgcn_rcpf(det);  // hardware reciprocal (1 ulp)
  if (!(t > tmin) || t > tbest) return false;
  t_out = t;
  return true;
}

// Ray/sphere in FP32 with the stable discriminant r^2 - |oc - b d|^2.
__device__ __forceinline__ bool sph_hit(const RayPre &r, F3 c, float rad, float tmin, float tbest,
                                        float &t_out) {
  F3 oc = r.o - c;
  float b = dot(oc, r.d);
  F3 f = oc - b * r.d;
  float disc = rad * rad - dot(f, f);
  if (disc < 0.f) return false;
  float sq = sqrtf(disc);
  float q = b > 0.f ? -(b + sq) : -(b - sq);  // the larger-magnitude root
  float t0 = q, t1 = (dot(oc, oc) - rad * rad) / q;
  if (t0 > t1) { float t = t0; t0 = t1; t1 = t; }
  float t = t0 > tmin ? t0 : t1;
  if (!(t > tmin) || t > tbest) return false;
  t_out = t;
  return true;
}

__device__ __forceinline__ void box2(const RayPre &r, float4 a, float4 b, float4 c, float tmin,
                                     float tmax, float &t0, float &t1, bool &h0, bool &h1) {
  float ox = r.o.x * r.inv.x, oy = r.o.y * r.inv.y, oz = r.o.z * r.inv.z;
  float l0x = a.x * r.inv.x - ox, h0x = a.y * r.inv.x - ox;
  float l0y = a.z * r.inv.y - oy, h0y = a.w * r.inv.y - oy;
  float l1x = b.x * r.inv.x - ox, h1x = b.y * r.inv.x - ox;
  float l1y = b.z * r.inv.y - oy, h1y = b.w * r.inv.y - oy;
  float l0z = c.x * r.inv.z - oz, h0z = c.y * r.inv.z - oz;
  float l1z = c.z * r.inv.z - oz, h1z = c.w * r.inv.z - oz;
  float n0 = fmaxf(fmaxf(fminf(l0x, h0x), fminf(l0y, h0y)), fmaxf(fminf(l0z, h0z), tmin));
  float f0 = fminf(fminf(fmaxf(l0x, h0x), fmaxf(l0y, h0y)), fminf(fmaxf(l0z, h0z), tmax));
  float n1 = fmaxf(fmaxf(fminf(l1x, h1x), fminf(l1y, h1y)), fmaxf(fminf(l1z, h1z), tmin));
  float f1 = fminf(fminf(fmaxf(l1x, h1x), fmaxf(l1y, h1y)), fminf(fmaxf(l1z, h1z), tmax));
  // slack of a few ulp so that rounding in the slabs never culls a hit
  h0 = n0 <= f0 * 1.0000004f; h1 = n1 <= f1 * 1.0000004f;
  t0 = n0; t1 = n1;
}

__device__ __forceinline__ void leaf_test(const RayPre &r, GF4 P, int32_t node, float tmin,
                                          int32_t exclude, Hit &best) {
  uint32_t v = (uint32_t)(~node);
  uint32_t first = v >> 3, cnt = (v & 7u) + 1u;
  for (uint32_t k = 0; k < cnt; ++k) {
    GF4 p = P + 3 * (size_t)(first + k);
    float4 p0 = ld4(p), p1 = ld4(p + 1);
    int32_t gid = __float_as_int(p0.w);
    if (gid == exclude) continue;
    float t;
    bool h;
    if (__float_as_int(p1.w) == 1) {
      h = sph_hit(r, f3(p0.x, p0.y, p0.z), p1.x, tmin, best.t, t);
    } else {
      float4 p2 = ld4(p + 2);
      h = tri_hit(r, f3(p0.x, p0.y, p0.z), f3(p1.x, p1.y, p1.z), f3(p2.x, p2.y, p2.z), tmin, best.t, t);
    }
    if (h) {
      // t <= best.t here; on a tie (rare: a shared edge) compare global ids
      bool take = t < best.t || best.prim < 0 || gid < __float_as_int(ld4(P + 3 * (size_t)best.prim).w);
      if (take) { best.t = t; best.prim = (int32_t)(first + k); }
    }
  }
}

// Traversal state of one lane: closest hit in (tmin, inf), ties to the
// lower global id, skipping the triangle `exclude`. The stack lives in LDS,
// one column per lane (consecutive entries `stride` ints apart, so lanes
// never share a bank).
struct Trav {
  RayPre r;
  float tmin;
  int32_t exclude;
  int32_t node;   // next node: >= 0 inner, < 0 leaf, kDone: finished
  int sp;
  Hit best;
};
constexpr int32_t kDone = 0x7FFFFFFF;

__device__ __forceinline__ void trav_init(Trav &T, F3 o, F3 d, float tmin, int32_t exclude, bool empty) {
  T.r = ray_pre(o, d);
  T.tmin = tmin * 1.0f + 0.0f;  // an arithmetic result: no canonicalisation in the loop
  T.exclude = exclude;
  T.node = empty ? kDone : 0;
  T.sp = 0;
  T.best.t = INFINITY;
  T.best.prim = -1;
}

// Traversal stack of one lane: the first kStackLds entries in LDS (lanes
// interleaved with stride `stride`), deeper ones in global memory (`spill`,
// one column per thread, entries `sstride` apart). Entries past the LDS
// part are rare: they need a path with that many pending far children.
typedef int32_t __attribute__((address_space(3))) *LdsI32;
typedef int32_t __attribute__((address_space(1))) *GlbI32;
typedef const v4f __attribute__((address_space(3))) *LF4;

// `nodes`: the first n_nodes BVH nodes (the top levels, stored first by the
// builder) copied to LDS by the workgroup, or n_nodes = 0.
struct Stack {
  LdsI32 lds;
  uint32_t stride;
  GlbI32 spill;
  uint32_t sstride;
  LF4 nodes;
  uint32_t n_nodes;
};

__device__ __forceinline__ void st_store(const Stack &S, int j, int32_t v) {
  if (j < kStackLds) S.lds[j * S.stride] = v;
  else S.spill[(size_t)(j - kStackLds) * S.sstride] = v;
}

__device__ __forceinline__ int32_t st_load(const Stack &S, int j) {
  return j < kStackLds ? S.lds[j * S.stride] : S.spill[(size_t)(j - kStackLds) * S.sstride];
}

__device__ __forceinline__ void push(const Stack &S, int &sp, int32_t v) {
  st_store(S, sp, v);
  ++sp;
}

__device__ __forceinline__ int32_t pop(const Stack &S, int &sp) {
  if (sp == 0) return kDone;
  --sp;
  return st_load(S, sp);
}

__device__ __forceinline__ float4 ld4l(LF4 p) {
  v4f v = *p;
  return make_float4(v.x, v.y, v.z, v.w);
}

// The four float4 of BVH node `node`: from LDS for the top levels.
__device__ __forceinline__ void load_node(const Stack &S, GF4 N, int32_t node, float4 &a, float4 &b, float4 &c,
                                          float4 &l) {
  if ((uint32_t)node < S.n_nodes) {
    a = ld4l(S.nodes + 4 * node); b = ld4l(S.nodes + 4 * node + 1);
    c = ld4l(S.nodes + 4 * node + 2); l = ld4l(S.nodes + 4 * node + 3);
  } else {
    a = ld4(N + 4 * node); b = ld4(N + 4 * node + 1); c = ld4(N + 4 * node + 2); l = ld4(N + 4 * node + 3);
  }
}

// Advance this lane by one round: descend inner nodes, postponing the first
// leaf reached and continuing with the next stack entry, until all but at
// most kTraceStragglers lanes of the wave hold a leaf or have nothing left to
// descend; then test the postponed leaf (Aila and Laine's speculative
// "while-while", which keeps lanes descending instead of idling while others
// look for a leaf; lanes still descending carry on next round). Leaves
// may be tested out of front-to-back order; the closest-hit and tie rules
// make the result independent of the order. COUNT adds node visits and
// primitive tests to nv / nt.
template <bool COUNT>
__device__ __forceinline__ void trav_step(Trav &T, GF4 N, GF4 P, const Stack &St, uint32_t &nv, uint32_t &nt) {
  int32_t node = T.node;
  int sp = T.sp;
  bool has_leaf = false;
  int32_t leaf = 0;
  for (;;) {
    if (node >= 0 && node != kDone) {
      if (COUNT) ++nv;
      float4 a, b, c, l4;
      load_node(St, N, node, a, b, c, l4);
      int32_t c0 = __float_as_int(l4.x), c1 = __float_as_int(l4.y);
      float t0, t1;
      bool h0, h1;
      box2(T.r, a, b, c, T.tmin, T.best.t, t0, t1, h0, h1);
      if (h0 && h1) {
        bool first0 = t0 <= t1;
        push(St, sp, first0 ? c1 : c0);
        node = first0 ? c0 : c1;
      } else if (h0) {
        node = c0;
      } else if (h1) {
        node = c1;
      } else {
        node = pop(St, sp);
      }
    }
    if (node < 0 && !has_leaf) {  // postpone the leaf, keep descending
      has_leaf = true;
      leaf = node;
      node = pop(St, sp);
    }
    bool ready = has_leaf || node == kDone || node < 0;
    // leave the descent once at most kTraceStragglers lanes are still
    // looking for a leaf (waiting for all of them leaves most of the wave
    // idle); the stragglers resume where they are in the next step
    if (__popcll(__ballot(!ready)) <= kTraceStragglers) break;
  }
  if (has_leaf) {
    if (COUNT) nt += ((uint32_t)(~leaf) & 7u) + 1u;
    leaf_test(T.r, P, leaf, T.tmin, T.exclude, T.best);
  } else if (node < 0) {
    if (COUNT) nt += ((uint32_t)(~node) & 7u) + 1u;
    leaf_test(T.r, P, node, T.tmin, T.exclude, T.best);
    node = pop(St, sp);
  }
  T.node = node;
  T.sp = sp;
}

// ------------------------------------------------------------------ FP64 refinement
// Exact-to-FP64 distance along (o, d) to the plane of the triangle chosen by
// the FP32 traversal, from its precomputed FP64 plane n.x = c: the optical
// path length of the coherent prefix uses this t.
__device__ __forceinline__ double tri_t64(double4 pl, D3 o, D3 d) {
  return (pl.w - (pl.x * o.x + pl.y * o.y + pl.z * o.z)) / (pl.x * d.x + pl.y * d.y + pl.z * d.z);
}

__device__ __forceinline__ double sph_t64(double4 s, D3 o, D3 d, double tmin) {
  D3 c = {s.x, s.y, s.z};
  double rad = s.w;
  D3 oc = o - c;
  double b = dot(oc, d);
  double cc = dot(oc, oc) - rad * rad;
  double disc = b * b - cc;
  double sq = sqrt(disc > 0 ? disc : 0.0);
  double t0 = -b - sq, t1 = -b + sq;
  return t0 > tmin ? t0 : t1;
}

// ------------------------------------------------------------------ BSDFs
// Orthonormal basis around n (Duff et al., JCGT 2017).
__device__ __forceinline__ void onb(F3 n, F3 &b1, F3 &b2) {
  float sign = copysignf(1.0f, n.z);
  float a = -1.0f / (sign + n.z);
  float b = n.x * n.y * a;
  b1 = f3(1.0f + sign * n.x * n.x * a, sign * b, -sign * n.x);
  b2 = f3(b, sign + n.y * n.y * a, -n.y);
}

__device__ __forceinline__ F3 reflect(F3 d, F3 n) { return d - (2.0f * dot(d, n)) * n; }
__device__ __forceinline__ D3 reflect(D3 d, D3 n) { return d - (2.0 * dot(d, n)) * n; }

// Unpolarised Fresnel reflectance of a dielectric interface (1 for total
// internal reflection); FP64 so that the lobe choice matches exactly.
__device__ __forceinline__ double fresnel64(double cos_i, double eta_i, double eta_t, double &cos_t) {
  double sin_i2 = fmax(0.0, 1.0 - cos_i * cos_i);
  double sin_t = eta_i / eta_t * sqrt(sin_i2);
  if (sin_t >= 1.0) { cos_t = 0.0; return 1.0; }
  cos_t = sqrt(fmax(0.0, 1.0 - sin_t * sin_t));
  double rs = (eta_i * cos_i - eta_t * cos_t) / (eta_i * cos_i + eta_t * cos_t);
  double rp = (eta_t * cos_i - eta_i * cos_t) / (eta_t * cos_i + eta_i * cos_t);
  return 0.5 * (rs * rs + rp * rp);
}

struct Lobe { F3 d; float w; uint32_t ev; bool delta; };

// GGX visible-normal sample (Heitz, JCGT 2018) in the local frame (z up).
__device__ __forceinline__ F3 vndf_local(F3 V, float a, float u1, float u2) {
  F3 Vh = normalize(f3(a * V.x, a * V.y, V.z));
  float lensq = Vh.x * Vh.x + Vh.y * Vh.y;
  F3 T1 = lensq > 0.f ? (1.0f / sqrtf(lensq)) * f3(-Vh.y, Vh.x, 0.f) : f3(1.f, 0.f, 0.f);
  F3 T2 = cross(Vh, T1);
  float r = sqrtf(u1), s, c;
  sincospif(2.0f * u2, &s, &c);
  float t1 = r * c, t2 = r * s;
  float sh = 0.5f * (1.0f + Vh.z);
  t2 = (1.0f - sh) * sqrtf(fmaxf(0.f, 1.f - t1 * t1)) + sh * t2;
  F3 Nh = t1 * T1 + t2 * T2 + sqrtf(fmaxf(0.f, 1.f - t1 * t1 - t2 * t2)) * Vh;
  return normalize(f3(a * Nh.x, a * Nh.y, fmaxf(0.f, Nh.z)));
}

__device__ __forceinline__ float smith_g1f(F3 w, float a) {
  return 2.0f * w.z / (w.z + sqrtf(a * a * (w.x * w.x + w.y * w.y) + w.z * w.z));
}

// Principled reflectance in FP32 (Burley 2012, metallic-roughness core):
// Burley diffuse weighted 1 - metallic; GGX specular, alpha = roughness^2,
// Schlick F0 = (1 - metallic) 0.08 specular + metallic base; GTR1 clearcoat
// (alpha 0.1 (1 - gloss) + 0.001 gloss, F0 0.04, Smith alpha 0.25) weighted
// 0.25 clearcoat. Lobes are sampled with probability proportional to
// (1 - metallic, 1, 0.25 clearcoat); f cos and the combined pdf for local
// V, L (z = facing normal).
struct BsdfEval { float fcos, pdf; };
__device__ __forceinline__ BsdfEval principled_eval(const MaterialDev &m, float base, F3 V, F3 L) {
  BsdfEval e{0.f, 0.f};
  if (L.z <= 0.f || V.z <= 0.f) return e;
  const float inv_pi = 0.318309886183790672f;
  const float r = m.rough, a = r * r;
  F3 H = normalize(V + L);
  const float vh = fmaxf(0.f, dot(V, H));
  const float x = 1.0f - vh, x2 = x * x, schlick = x2 * x2 * x;
  const float fd90 = 0.5f + 2.0f * r * vh * vh;
  const float xl = 1.0f - L.z, xl2 = xl * xl, xv = 1.0f - V.z, xv2 = xv * xv;
  const float fdiff = (1.0f - m.metallic) * base * inv_pi * (1.0f + (fd90 - 1.0f) * xl2 * xl2 * xl) *
                      (1.0f + (fd90 - 1.0f) * xv2 * xv2 * xv);
  const float f0 = (1.0f - m.metallic) * 0.08f * m.specular + m.metallic * base;
  const float a2 = a * a, k = H.z * H.z * (a2 - 1.0f) + 1.0f;
  const float D = a2 * inv_pi / (k * k);
  const float g1v = smith_g1f(V, a);
  const float fspec = (f0 + (1.0f - f0) * schlick) * D * g1v * smith_g1f(L, a) / (4.0f * V.z * L.z);
  const float ac = 0.1f * (1.0f - m.clearcoat_gloss) + 0.001f * m.clearcoat_gloss, ac2 = ac * ac;
  const float Dc = (ac2 - 1.0f) * inv_pi / (logf(ac2) * (1.0f + (ac2 - 1.0f) * H.z * H.z));
  const float fcc = 0.25f * m.clearcoat * (0.04f + 0.96f * schlick) * Dc * smith_g1f(V, 0.25f) *
                    smith_g1f(L, 0.25f) / (4.0f * V.z * L.z);
  const float wd = 1.0f - m.metallic, wc = 0.25f * m.clearcoat, sum = wd + 1.0f + wc;
  e.pdf = (wd * L.z * inv_pi + g1v * D / (4.0f * V.z) + (vh > 0.f ? wc * Dc * H.z / (4.0f * vh) : 0.f)) / sum;
  e.fcos = (fdiff + fspec + fcc) * L.z;
  return e;
}

__device__ __forceinline__ F3 principled_sample(const MaterialDev &m, F3 V, float u0, float u1, float u2,
                                                uint32_t &lobe) {
  const float wd = 1.0f - m.metallic, wc = 0.25f * m.clearcoat, sum = wd + 1.0f + wc;
  const float xs = u0 * sum;
  lobe = xs < wd ? 0u : (xs < wd + 1.0f ? 1u : 2u);
  if (lobe == 0u) {
    float r = sqrtf(u1), s, c;
    sincospif(2.0f * u2, &s, &c);
    return f3(r * c, r * s, sqrtf(fmaxf(0.f, 1.f - u1)));
  }
  F3 H;
  if (lobe == 1u) {
    H = vndf_local(V, m.rough * m.rough, u1, u2);
  } else {
    const float ac = 0.1f * (1.0f - m.clearcoat_gloss) + 0.001f * m.clearcoat_gloss, ac2 = ac * ac;
    const float ct = sqrtf(fmaxf(0.f, (1.0f - powf(ac2, 1.0f - u1)) / (1.0f - ac2)));
    const float st = sqrtf(fmaxf(0.f, 1.0f - ct * ct));
    float s, c;
    sincospif(2.0f * u2, &s, &c);
    H = f3(st * c, st * s, ct);
  }
  return (2.0f * dot(V, H)) * H - V;
}

// One lobe sample in FP32 for the incoherent tail (Lambert cosine, GGX
// visible normals with weight F_schlick * G1(L), mirror, dielectric with
// Fresnel choice and (eta_i/eta_t)^2 on refraction; with EXT also the
// principled lobes, kept out of the base shading kernel's registers).
template <bool EXT>
__device__ __forceinline__ Lobe sample_lobe(const MaterialDev &m, uint32_t comp, F3 d_in, F3 ng,
                                            float u0, float u1, float u2) {
  Lobe L;
  L.w = 0.f; L.delta = false; L.ev = 0; L.d = d_in;
  float dn = dot(d_in, ng);
  F3 nf = dn < 0.f ? ng : (-1.0f) * ng;
  float rgb = comp == 0 ? m.rgb[0] : (comp == 1 ? m.rgb[1] : m.rgb[2]);
  if (m.type == HPT_LAMBERT) {
    F3 b1, b2;
    onb(nf, b1, b2);
    float r = sqrtf(u1), s, c;
    sincospif(2.0f * u2, &s, &c);
    float z = sqrtf(fmaxf(0.f, 1.f - u1));
    L.d = (r * c) * b1 + (r * s) * b2 + z * nf;
    L.w = rgb; L.ev = EV_LAMBERT;
  } else if (m.type == HPT_MIRROR) {
    L.d = reflect(d_in, nf); L.w = 1.f; L.ev = EV_MIRROR; L.delta = true;
  } else if (m.type == HPT_DIELECTRIC) {
    bool entering = dn < 0.f;
    double eta_i = entering ? 1.0 : m.ior, eta_t = entering ? m.ior : 1.0;
    double cos_t;
    double F = fresnel64(fabs((double)dn), eta_i, eta_t, cos_t);
    L.delta = true;
    if ((double)u0 < F) {
      L.d = reflect(d_in, nf); L.w = 1.f; L.ev = EV_DIEL_REFL;
    } else {
      float e = (float)(eta_i / eta_t);
      float ci = fabsf(dn);
      L.d = normalize(e * d_in + (e * ci - (float)cos_t) * nf);
      L.w = e * e; L.ev = EV_DIEL_REFR;
    }
  } else if (EXT && m.type == HPT_PRINCIPLED) {
    F3 b1, b2;
    onb(nf, b1, b2);
    F3 wo = (-1.0f) * d_in;
    F3 V = f3(dot(wo, b1), dot(wo, b2), dot(wo, nf));
    uint32_t lobe;
    F3 Lw = principled_sample(m, V, u0, u1, u2, lobe);
    L.ev = EV_PRIN_DIFFUSE + lobe;
    if (Lw.z <= 0.f || V.z <= 0.f) { L.w = 0.f; L.ev = EV_ABSORB; return L; }
    BsdfEval e = principled_eval(m, rgb, V, Lw);
    L.w = e.pdf > 0.f ? e.fcos / e.pdf : 0.f;
    L.d = normalize(Lw.x * b1 + Lw.y * b2 + Lw.z * nf);
  } else if (m.type == HPT_GGX) {
    F3 b1, b2;
    onb(nf, b1, b2);
    F3 wo = (-1.0f) * d_in;
    F3 V = f3(dot(wo, b1), dot(wo, b2), dot(wo, nf));
    float a = m.rough;
    F3 Vh = normalize(f3(a * V.x, a * V.y, V.z));
    float lensq = Vh.x * Vh.x + Vh.y * Vh.y;
    F3 T1 = lensq > 0.f ? (1.0f / sqrtf(lensq)) * f3(-Vh.y, Vh.x, 0.f) : f3(1.f, 0.f, 0.f);
    F3 T2 = cross(Vh, T1);
    float r = sqrtf(u1), s, c;
    sincospif(2.0f * u2, &s, &c);
    float t1 = r * c, t2 = r * s;
    float sh = 0.5f * (1.0f + Vh.z);
    t2 = (1.0f - sh) * sqrtf(fmaxf(0.f, 1.f - t1 * t1)) + sh * t2;
    F3 Nh = t1 * T1 + t2 * T2 + sqrtf(fmaxf(0.f, 1.f - t1 * t1 - t2 * t2)) * Vh;
    F3 M = normalize(f3(a * Nh.x, a * Nh.y, fmaxf(0.f, Nh.z)));
    float vm = dot(V, M);
    F3 Lw = (2.0f * vm) * M - V;
    L.ev = EV_GGX;
    if (Lw.z <= 0.f || V.z <= 0.f) { L.w = 0.f; L.ev = EV_ABSORB; return L; }
    float x = 1.0f - fmaxf(0.f, vm);
    float x2 = x * x;
    float F = rgb + (1.0f - rgb) * (x2 * x2 * x);
    float g1 = 2.0f * Lw.z / (Lw.z + sqrtf(a * a * (Lw.x * Lw.x + Lw.y * Lw.y) + Lw.z * Lw.z));
    L.w = F * g1;
    L.d = normalize(Lw.x * b1 + Lw.y * b2 + Lw.z * nf);
  }
  return L;
}

// f cos and the pdf (solid angle) with which sample_lobe draws the direction
// wl leaving a non-delta surface (cosines against the normal facing the
// incoming ray d_in). GGX: f cos = F D G1(V) G1(L) / (4 V.z) and
// pdf = G1(V) D / (4 V.z), whose ratio is the sampling weight F G1(L).
template <bool EXT>
__device__ __forceinline__ BsdfEval eval_lobe(const MaterialDev &m, uint32_t comp, F3 d_in, F3 ng, F3 wl) {
  BsdfEval e{0.f, 0.f};
  F3 nf = dot(d_in, ng) < 0.f ? ng : (-1.0f) * ng;
  float c = dot(wl, nf);
  if (c <= 0.f) return e;
  float rgb = comp == 0 ? m.rgb[0] : (comp == 1 ? m.rgb[1] : m.rgb[2]);
  const float inv_pi = 0.318309886183790672f;
  if (m.type == HPT_LAMBERT) {
    e.fcos = rgb * c * inv_pi;
    e.pdf = c * inv_pi;
  } else if (EXT && m.type == HPT_PRINCIPLED) {
    F3 b1, b2;
    onb(nf, b1, b2);
    F3 wo = (-1.0f) * d_in;
    e = principled_eval(m, rgb, f3(dot(wo, b1), dot(wo, b2), dot(wo, nf)), f3(dot(wl, b1), dot(wl, b2), c));
  } else if (m.type == HPT_GGX) {
    F3 b1, b2;
    onb(nf, b1, b2);
    F3 wo = (-1.0f) * d_in;
    F3 V = f3(dot(wo, b1), dot(wo, b2), dot(wo, nf));
    if (V.z <= 0.f) return e;
    F3 Lw = f3(dot(wl, b1), dot(wl, b2), c);
    F3 H = normalize(V + Lw);
    float a = m.rough, a2 = a * a;
    float k = H.z * H.z * (a2 - 1.0f) + 1.0f;
    float D = a2 * inv_pi / (k * k);
    float x = 1.0f - fmaxf(0.f, dot(V, H));
    float x2 = x * x;
    float F = rgb + (1.0f - rgb) * (x2 * x2 * x);
    float g1v = 2.0f * V.z / (V.z + sqrtf(a2 * (V.x * V.x + V.y * V.y) + V.z * V.z));
    float g1l = 2.0f * Lw.z / (Lw.z + sqrtf(a2 * (Lw.x * Lw.x + Lw.y * Lw.y) + Lw.z * Lw.z));
    e.pdf = g1v * D / (4.0f * V.z);
    e.fcos = e.pdf * F * g1l;
  }
  return e;
}

// Octahedral map of a unit direction to a bins x bins grid.
__device__ __forceinline__ uint32_t oct_bin(F3 w, uint32_t bins) {
  float s = fabsf(w.x) + fabsf(w.y) + fabsf(w.z);
  float px = w.x / s, py = w.y / s;
  if (w.z < 0.f) {
    float sx = px >= 0.f ? 1.f : -1.f, sy = py >= 0.f ? 1.f : -1.f;
    float nx = (1.f - fabsf(py)) * sx, ny = (1.f - fabsf(px)) * sy;
    px = nx; py = ny;
  }
  int bu = (int)floorf((px + 1.f) * 0.5f * (float)bins);
  int bv = (int)floorf((py + 1.f) * 0.5f * (float)bins);
  bu = min(max(bu, 0), (int)bins - 1);
  bv = min(max(bv, 0), (int)bins - 1);
  return (uint32_t)bv * bins + (uint32_t)bu;
}

__device__ __forceinline__ D3 oct_decode64(double u, double v) {
  double z = 1.0 - fabs(u) - fabs(v);
  double x = u, y = v;
  if (z < 0) {
    double sx = x >= 0 ? 1.0 : -1.0, sy = y >= 0 ? 1.0 : -1.0;
    double nx = (1.0 - fabs(y)) * sx, ny = (1.0 - fabs(x)) * sy;
    x = nx; y = ny;
  }
  return normalize(D3{x, y, z});
}

}  // namespace hpt
