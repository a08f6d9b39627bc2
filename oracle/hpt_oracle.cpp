// FP64 CPU oracle for the wave path tracer -- TEST INFRASTRUCTURE ONLY.
//
// Only tests, the smoke check and the CPU-baseline leg of the benchmark may
// load this library. The GPU library never links, calls or reads it, and it
// shares no source with the GPU library.
//
// It computes, slowly and plainly in double precision, the Monte Carlo
// estimator of the paper (HoloPathTracer, ACM TOG 45(4) 2026):
//   * rays leave each recording-plane pixel inside the recordable cone
//     sin(theta) <= lambda/(2d)                         (Sec. 4.1, Sec. 4.2)
//   * they are moved to world space by the inverse of T (Eq. 3)
//   * delta lobes (mirror, ideal refraction) continue the coherent path and
//     add n_i * L_i to the optical path length          (Sec. 4.2, OPL sum)
//   * the first non-delta hit is the real image point P; incoherent
//     radiance rays from P give the amplitude A = sqrt(average radiance)
//     (Sec. 4 stage s5, Eq. 1)
//   * the virtual image point P' = O + d_OPL v is mapped to Q = T P'
//     (Sec. 4.2), and the contribution A exp(i(k r + phi_m(Q))) is added to
//     every frame m (Eq. 5), phi_m = arg r_m taken from the band-limited
//     random fields of Eq. 4 (Sec. 4.3, Path Reuse).
// Readings where the paper is silent (weights, sampling density, bounce
// semantics, the radiance cache layout) are restated at each function below.
//
// Pins (tests/test_oracle_pins.py): Philox known answers; closed-form sphere
// and triangle hits; BVH == brute force; Fresnel textbook values; Lambert and
// GGX-VNDF sample densities; RS integral of Eq. 2 by quadrature (patch,
// mirror image, wide-cone plane); slab OPL by Snell; radiance theorem in
// glass; white furnace; GGX weight by quadrature; Eq. 3 rotation invariance;
// Eq. 4 by brute-force DFT and spectrum support; Path Reuse invariants.
// Parity unpinned: the radiance cache entries beyond the furnace case (the
// paper leaves the cache to its supplement; the grid/bin layout is a
// reading), and the path signature hash (bookkeeping, not the method).
//
// Build: g++ -O2 -std=c++17 -fopenmp -shared -fPIC (no fast-math).

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <omp.h>
#include <unordered_map>
#include <vector>

namespace {

// ------------------------------------------------------------------ Philox
// Philox4x32-10, Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11: ten rounds of two 32x32->64 multiplies; the key is
// bumped by the Weyl constants between rounds.
inline void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    uint64_t p0 = (uint64_t)M0 * c0;
    uint64_t p1 = (uint64_t)M1 * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// 24-bit uniform in [0,1): exactly representable in float and double.
inline double u01(uint32_t w) { return (double)(w >> 8) * (1.0 / 16777216.0); }

// Streams of the counter-based generator.
enum { STREAM_PATH = 0, STREAM_CACHE = 2, STREAM_GRF = 3 };

struct Uniforms { double u[4]; };

// Path stream: counter = (pixel, sample, interaction<<8 | tail, comp<<16 | stream).
inline Uniforms path_uniforms(uint64_t seed, uint32_t pixel, uint32_t sample, uint32_t b,
                              uint32_t comp) {
  uint32_t ctr[4] = {pixel, sample, b << 8, (comp << 16) | STREAM_PATH};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  philox4x32_10(ctr, key, w);
  Uniforms r;
  for (int i = 0; i < 4; ++i) r.u[i] = u01(w[i]);
  return r;
}

// ------------------------------------------------------------------ vectors
struct V3 { double x, y, z; };
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
inline double length(V3 a) { return std::sqrt(dot(a, a)); }
inline V3 normalize(V3 a) { return (1.0 / length(a)) * a; }
inline double comp_of(V3 a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }

// ------------------------------------------------------------------ hashing
// Path signature: 64-bit FNV-1a over 32-bit words (one word per step).
const uint64_t FNV_OFFSET = 0xcbf29ce484222325ull, FNV_PRIME = 0x100000001b3ull;
inline void sig_add(uint64_t &h, uint32_t w) { h ^= (uint64_t)w; h *= FNV_PRIME; }

// Lobe / event codes recorded in the signature.
enum { EV_MIRROR = 1, EV_DIEL_REFL = 2, EV_DIEL_REFR = 3, EV_LAMBERT = 4, EV_GGX = 5,
       EV_ABSORB = 6, EV_EMIT = 7, EV_IMAGE_POINT = 8, EV_PRIN_DIFFUSE = 9, EV_PRIN_SPECULAR = 10,
       EV_PRIN_CLEARCOAT = 11 };
// Termination kinds.
enum { K_NONE = 0, K_ESCAPE_PREFIX = 1, K_MAXB_PREFIX = 2, K_EMITTER = 3, K_ENV = 4,
       K_MAXB_TAIL = 5, K_CACHE = 6, K_ABSORBED = 7 };

enum { LAMBERT = 0, GGX = 1, MIRROR = 2, DIELECTRIC = 3, EMITTER = 4, PRINCIPLED = 5 };

// ------------------------------------------------------------------ scene
struct Material {
  int type;
  double rgb[3], rough, ior, emit[3];
  double metallic, specular, clearcoat, clearcoat_gloss;   // PRINCIPLED
};

struct Box { V3 lo, hi; };

struct Node {            // binary BVH node (oracle's own, median split)
  Box box;
  int left, right;       // children (internal) or -1
  int first, count;      // primitive range (leaf)
};

// Emitter triangle for next-event estimation (unit normal n along
// (v1 - v0) x (v2 - v0), the side it emits on).
struct Light { V3 v0, v1, v2, n; double area; int mat; };

struct Scene {
  int n_sph = 0, n_tri = 0;
  std::vector<V3> sc;            // sphere centres
  std::vector<double> sr;        // sphere radii
  std::vector<V3> tv;            // triangle vertices, 3 per triangle
  std::vector<int> prim_mat;     // material per global id
  std::vector<Material> mats;
  double env[3];
  std::vector<Node> nodes;
  std::vector<int> order;        // primitive ids in leaf order
  Box bounds;
  std::vector<Light> lights;     // emitter triangles in id order
  std::vector<double> light_cdf; // running sum of their areas
  double light_area = 0.0;
  std::vector<V3> pt_pos;        // point emitters: position (world space)
  std::vector<V3> pt_amp;        // and amplitude per colour component
};

struct Hit { double t; int gid; };

Box prim_box(const Scene &S, int gid) {
  Box b;
  if (gid < S.n_sph) {
    V3 c = S.sc[gid]; double r = S.sr[gid];
    b.lo = {c.x - r, c.y - r, c.z - r}; b.hi = {c.x + r, c.y + r, c.z + r};
  } else {
    int i = gid - S.n_sph;
    V3 a = S.tv[3 * i], q = S.tv[3 * i + 1], c = S.tv[3 * i + 2];
    b.lo = {std::min({a.x, q.x, c.x}), std::min({a.y, q.y, c.y}), std::min({a.z, q.z, c.z})};
    b.hi = {std::max({a.x, q.x, c.x}), std::max({a.y, q.y, c.y}), std::max({a.z, q.z, c.z})};
  }
  return b;
}

Box merge(Box a, Box b) {
  return {{std::min(a.lo.x, b.lo.x), std::min(a.lo.y, b.lo.y), std::min(a.lo.z, b.lo.z)},
          {std::max(a.hi.x, b.hi.x), std::max(a.hi.y, b.hi.y), std::max(a.hi.z, b.hi.z)}};
}

// Median split on the longest axis of the centroid bounds; leaves hold <= 4.
int build_node(Scene &S, std::vector<Box> &pb, std::vector<V3> &pc, int first, int count) {
  Node nd;
  nd.box = pb[S.order[first]];
  for (int i = 1; i < count; ++i) nd.box = merge(nd.box, pb[S.order[first + i]]);
  // pad so that rounding in the slab test can never cull a true hit
  double ext = std::max({nd.box.hi.x - nd.box.lo.x, nd.box.hi.y - nd.box.lo.y,
                         nd.box.hi.z - nd.box.lo.z});
  double pad = 1e-12 + 1e-9 * ext;
  nd.box.lo = nd.box.lo - V3{pad, pad, pad};
  nd.box.hi = nd.box.hi + V3{pad, pad, pad};
  int id = (int)S.nodes.size();
  S.nodes.push_back(nd);
  if (count <= 4) {
    S.nodes[id].left = S.nodes[id].right = -1;
    S.nodes[id].first = first; S.nodes[id].count = count;
    return id;
  }
  V3 lo = pc[S.order[first]], hi = lo;
  for (int i = 1; i < count; ++i) {
    V3 c = pc[S.order[first + i]];
    lo = {std::min(lo.x, c.x), std::min(lo.y, c.y), std::min(lo.z, c.z)};
    hi = {std::max(hi.x, c.x), std::max(hi.y, c.y), std::max(hi.z, c.z)};
  }
  V3 e = hi - lo;
  int axis = (e.x >= e.y && e.x >= e.z) ? 0 : (e.y >= e.z ? 1 : 2);
  int mid = count / 2;
  std::nth_element(S.order.begin() + first, S.order.begin() + first + mid,
                   S.order.begin() + first + count, [&](int a, int b) {
                     double ca = comp_of(pc[a], axis), cb = comp_of(pc[b], axis);
                     return ca < cb || (ca == cb && a < b);
                   });
  int l = build_node(S, pb, pc, first, mid);
  int r = build_node(S, pb, pc, first + mid, count - mid);
  S.nodes[id].left = l; S.nodes[id].right = r;
  S.nodes[id].first = first; S.nodes[id].count = 0;
  return id;
}

// Ray-sphere: smallest root of |o + t d - c|^2 = r^2 with t > tmin (|d| = 1).
bool hit_sphere(V3 c, double r, V3 o, V3 d, double tmin, double &t) {
  V3 oc = o - c;
  double b = dot(oc, d);
  double cc = dot(oc, oc) - r * r;
  double disc = b * b - cc;
  if (disc < 0) return false;
  double sq = std::sqrt(disc);
  double t0 = -b - sq, t1 = -b + sq;
  if (t0 > tmin) { t = t0; return true; }
  if (t1 > tmin) { t = t1; return true; }
  return false;
}

// Ray-triangle (Moller-Trumbore), two-sided, edges inclusive, t > tmin.
bool hit_triangle(V3 v0, V3 v1, V3 v2, V3 o, V3 d, double tmin, double &t) {
  V3 e1 = v1 - v0, e2 = v2 - v0;
  V3 p = cross(d, e2);
  double det = dot(e1, p);
  if (det == 0.0) return false;
  double inv = 1.0 / det;
  V3 s = o - v0;
  double u = dot(s, p) * inv;
  if (u < 0.0 || u > 1.0) return false;
  V3 q = cross(s, e1);
  double v = dot(d, q) * inv;
  if (v < 0.0 || u + v > 1.0) return false;
  double tt = dot(e2, q) * inv;
  if (!(tt > tmin)) return false;
  t = tt;
  return true;
}

inline void test_prim(const Scene &S, int gid, V3 o, V3 d, double tmin, int exclude, Hit &best) {
  if (gid == exclude) return;
  double t;
  bool h;
  if (gid < S.n_sph) h = hit_sphere(S.sc[gid], S.sr[gid], o, d, tmin, t);
  else {
    int i = gid - S.n_sph;
    h = hit_triangle(S.tv[3 * i], S.tv[3 * i + 1], S.tv[3 * i + 2], o, d, tmin, t);
  }
  if (h && (t < best.t || (t == best.t && gid < best.gid))) { best.t = t; best.gid = gid; }
}

// Slab test; an axis with d == 0 only checks that o lies inside the slab.
bool hit_box(const Box &b, V3 o, V3 d, double tmax_incl, double &tnear) {
  double t0 = -INFINITY, t1 = INFINITY;
  for (int a = 0; a < 3; ++a) {
    double oa = comp_of(o, a), da = comp_of(d, a);
    double lo = comp_of(b.lo, a), hi = comp_of(b.hi, a);
    if (da == 0.0) {
      if (oa < lo || oa > hi) return false;
      continue;
    }
    double ta = (lo - oa) / da, tb = (hi - oa) / da;
    if (ta > tb) std::swap(ta, tb);
    t0 = std::max(t0, ta); t1 = std::min(t1, tb);
  }
  tnear = t0;
  return t0 <= t1 && t1 >= 0.0 && t0 <= tmax_incl;
}

// Closest hit = minimum t over all primitives, ties to the lower id. `exclude`
// is the previous triangle (spheres are never excluded; t_min handles them).
Hit closest_hit(const Scene &S, V3 o, V3 d, double tmin, int exclude, bool brute) {
  Hit best{INFINITY, -1};
  if (brute || S.nodes.empty()) {
    for (int g = 0; g < S.n_sph + S.n_tri; ++g) test_prim(S, g, o, d, tmin, exclude, best);
    return best;
  }
  int stack[128];
  int sp = 0;
  stack[sp++] = 0;
  while (sp) {
    const Node &n = S.nodes[stack[--sp]];
    double tn;
    if (!hit_box(n.box, o, d, best.t, tn)) continue;
    if (n.left < 0) {
      for (int i = 0; i < n.count; ++i) test_prim(S, S.order[n.first + i], o, d, tmin, exclude, best);
    } else {
      stack[sp++] = n.left;
      stack[sp++] = n.right;
    }
  }
  return best;
}

V3 geom_normal(const Scene &S, int gid, V3 x) {
  if (gid < S.n_sph) return (1.0 / S.sr[gid]) * (x - S.sc[gid]);
  int i = gid - S.n_sph;
  return normalize(cross(S.tv[3 * i + 1] - S.tv[3 * i], S.tv[3 * i + 2] - S.tv[3 * i]));
}

// ------------------------------------------------------------------ BSDFs
// Orthonormal basis around unit n (Duff et al., "Building an Orthonormal
// Basis, Revisited", JCGT 2017).
void onb(V3 n, V3 &b1, V3 &b2) {
  double sign = std::copysign(1.0, n.z);
  double a = -1.0 / (sign + n.z);
  double b = n.x * n.y * a;
  b1 = {1.0 + sign * n.x * n.x * a, sign * b, -sign * n.x};
  b2 = {b, sign + n.y * n.y * a, -n.y};
}

V3 reflect(V3 d, V3 n) { return d - (2.0 * dot(d, n)) * n; }

// Exact unpolarised Fresnel reflectance for a dielectric interface; returns 1
// for total internal reflection. cos_i > 0 is the incidence cosine.
double fresnel_dielectric(double cos_i, double eta_i, double eta_t, double &cos_t) {
  double sin_i2 = std::max(0.0, 1.0 - cos_i * cos_i);
  double sin_t = eta_i / eta_t * std::sqrt(sin_i2);
  if (sin_t >= 1.0) { cos_t = 0.0; return 1.0; }
  cos_t = std::sqrt(std::max(0.0, 1.0 - sin_t * sin_t));
  double rs = (eta_i * cos_i - eta_t * cos_t) / (eta_i * cos_i + eta_t * cos_t);
  double rp = (eta_t * cos_i - eta_i * cos_t) / (eta_t * cos_i + eta_i * cos_t);
  return 0.5 * (rs * rs + rp * rp);
}

// Cosine-weighted hemisphere around n: radius sqrt(u1), angle 2 pi u2.
V3 sample_lambert(V3 n, double u1, double u2) {
  V3 b1, b2;
  onb(n, b1, b2);
  double r = std::sqrt(u1), ph = 2.0 * M_PI * u2;
  double z = std::sqrt(std::max(0.0, 1.0 - u1));
  return (r * std::cos(ph)) * b1 + (r * std::sin(ph)) * b2 + z * n;
}

// GGX visible-normal sampling (Heitz, "Sampling the GGX Distribution of
// Visible Normals", JCGT 2018) in the local frame of the normal (z up).
V3 sample_vndf_local(V3 V, double alpha, double u1, double u2) {
  V3 Vh = normalize(V3{alpha * V.x, alpha * V.y, V.z});
  double lensq = Vh.x * Vh.x + Vh.y * Vh.y;
  V3 T1 = lensq > 0 ? (1.0 / std::sqrt(lensq)) * V3{-Vh.y, Vh.x, 0.0} : V3{1.0, 0.0, 0.0};
  V3 T2 = cross(Vh, T1);
  double r = std::sqrt(u1), ph = 2.0 * M_PI * u2;
  double t1 = r * std::cos(ph), t2 = r * std::sin(ph);
  double s = 0.5 * (1.0 + Vh.z);
  t2 = (1.0 - s) * std::sqrt(std::max(0.0, 1.0 - t1 * t1)) + s * t2;
  V3 Nh = t1 * T1 + t2 * T2 + std::sqrt(std::max(0.0, 1.0 - t1 * t1 - t2 * t2)) * Vh;
  return normalize(V3{alpha * Nh.x, alpha * Nh.y, std::max(0.0, Nh.z)});
}

// Smith masking for GGX of a unit local direction w (z up).
double smith_g1(V3 w, double alpha) {
  double z2 = w.z * w.z;
  return 2.0 * w.z / (w.z + std::sqrt(alpha * alpha * (w.x * w.x + w.y * w.y) + z2));
}

// Principled reflectance (Burley, "Physically-Based Shading at Disney",
// SIGGRAPH 2012 course; its metallic-roughness core): Burley diffuse weighted
// 1 - metallic; GGX specular, alpha = roughness^2, Schlick F0 =
// (1 - metallic) 0.08 specular + metallic base, Smith masking G1(V) G1(L);
// GTR1 clearcoat, alpha = 0.1 (1 - gloss) + 0.001 gloss, F0 = 0.04, Smith
// masking with alpha 0.25, weighted 0.25 clearcoat. Sampling picks a lobe
// with probability proportional to (1 - metallic, 1, 0.25 clearcoat) and
// weights by the full f cos over the combined pdf (one-sample MIS). V, L in
// the local frame of the facing normal (z up).
struct PrinLobes { double wd, ws, wc, sum; };
PrinLobes prin_lobes(const Material &m) {
  PrinLobes p{1.0 - m.metallic, 1.0, 0.25 * m.clearcoat, 0.0};
  p.sum = p.wd + p.ws + p.wc;
  return p;
}

double gtr1(double cos_h, double a) {
  double a2 = a * a;
  return (a2 - 1.0) / (M_PI * std::log(a2) * (1.0 + (a2 - 1.0) * cos_h * cos_h));
}

struct PrinEval { double fcos, pdf; };
PrinEval principled_eval(const Material &m, int comp, V3 V, V3 L) {
  if (L.z <= 0.0 || V.z <= 0.0) return {0.0, 0.0};
  const double r = m.rough, a = r * r;
  V3 H = normalize(V + L);
  double vh = std::max(0.0, dot(V, H));
  double schlick = std::pow(1.0 - vh, 5.0);
  double fd90 = 0.5 + 2.0 * r * vh * vh;
  double fdiff = (1.0 - m.metallic) * m.rgb[comp] / M_PI * (1.0 + (fd90 - 1.0) * std::pow(1.0 - L.z, 5.0)) *
                 (1.0 + (fd90 - 1.0) * std::pow(1.0 - V.z, 5.0));
  double f0 = (1.0 - m.metallic) * 0.08 * m.specular + m.metallic * m.rgb[comp];
  double a2 = a * a, k = H.z * H.z * (a2 - 1.0) + 1.0;
  double D = a2 / (M_PI * k * k);
  double g1v = smith_g1(V, a);
  double fspec = (f0 + (1.0 - f0) * schlick) * D * g1v * smith_g1(L, a) / (4.0 * V.z * L.z);
  double ac = 0.1 * (1.0 - m.clearcoat_gloss) + 0.001 * m.clearcoat_gloss;
  double Dc = gtr1(H.z, ac);
  double fcc = 0.25 * m.clearcoat * (0.04 + 0.96 * schlick) * Dc * smith_g1(V, 0.25) * smith_g1(L, 0.25) /
               (4.0 * V.z * L.z);
  PrinLobes p = prin_lobes(m);
  double pdf = (p.wd * L.z / M_PI + p.ws * g1v * D / (4.0 * V.z) + (vh > 0.0 ? p.wc * Dc * H.z / (4.0 * vh) : 0.0)) /
               p.sum;
  return {(fdiff + fspec + fcc) * L.z, pdf};
}

// Lobe index (0 diffuse, 1 specular, 2 clearcoat) and the local direction
// drawn from it with u1, u2.
V3 principled_sample(const Material &m, V3 V, double u0, double u1, double u2, int &lobe) {
  PrinLobes p = prin_lobes(m);
  double x = u0 * p.sum;
  lobe = x < p.wd ? 0 : (x < p.wd + p.ws ? 1 : 2);
  if (lobe == 0) {
    double r = std::sqrt(u1), ph = 2.0 * M_PI * u2;
    return {r * std::cos(ph), r * std::sin(ph), std::sqrt(std::max(0.0, 1.0 - u1))};
  }
  V3 H;
  if (lobe == 1) {
    H = sample_vndf_local(V, m.rough * m.rough, u1, u2);
  } else {
    double ac = 0.1 * (1.0 - m.clearcoat_gloss) + 0.001 * m.clearcoat_gloss, ac2 = ac * ac;
    double ct = std::sqrt(std::max(0.0, (1.0 - std::pow(ac2, 1.0 - u1)) / (1.0 - ac2)));
    double st = std::sqrt(std::max(0.0, 1.0 - ct * ct)), ph = 2.0 * M_PI * u2;
    H = {st * std::cos(ph), st * std::sin(ph), ct};
  }
  return (2.0 * dot(V, H)) * H - V;
}

struct Sampled { V3 d; double w; int ev; bool delta; double eta_t; };

// One BSDF lobe sample at a surface. d_in: travel direction of the incoming
// ray; ng: geometric normal (outward for dielectrics); comp: colour channel.
// Lambert: weight albedo. GGX: VNDF around the direction back toward the
// previous vertex, weight F_schlick(V.m) * G1(L) (0 below the horizon).
// Mirror: weight 1. Dielectric: reflect with probability F (weight 1), else
// refract with weight (eta_i/eta_t)^2 (radiance scaling).
Sampled sample_bsdf(const Material &m, int comp, V3 d_in, V3 ng, const Uniforms &U,
                    double eta_cur) {
  Sampled s{{0, 0, 0}, 0.0, 0, false, eta_cur};
  V3 nf = dot(d_in, ng) < 0 ? ng : -1.0 * ng;   // normal facing the incoming side
  if (m.type == LAMBERT) {
    s.d = sample_lambert(nf, U.u[1], U.u[2]);
    s.w = m.rgb[comp]; s.ev = EV_LAMBERT;
  } else if (m.type == MIRROR) {
    s.d = reflect(d_in, nf); s.w = 1.0; s.ev = EV_MIRROR; s.delta = true;
  } else if (m.type == DIELECTRIC) {
    bool entering = dot(d_in, ng) < 0;
    double eta_i = entering ? 1.0 : m.ior, eta_t = entering ? m.ior : 1.0;
    double cos_i = std::fabs(dot(d_in, ng)), cos_t;
    double F = fresnel_dielectric(cos_i, eta_i, eta_t, cos_t);
    s.delta = true;
    if (U.u[0] < F) {
      s.d = reflect(d_in, nf); s.w = 1.0; s.ev = EV_DIEL_REFL;
    } else {
      double e = eta_i / eta_t;
      s.d = e * d_in + (e * cos_i - cos_t) * nf;
      s.d = normalize(s.d);
      s.w = e * e; s.ev = EV_DIEL_REFR; s.eta_t = eta_t;
    }
  } else if (m.type == PRINCIPLED) {
    V3 b1, b2;
    onb(nf, b1, b2);
    V3 wo = -1.0 * d_in;
    V3 V = {dot(wo, b1), dot(wo, b2), dot(wo, nf)};
    int lobe;
    V3 L = principled_sample(m, V, U.u[0], U.u[1], U.u[2], lobe);
    s.ev = EV_PRIN_DIFFUSE + lobe;
    if (L.z <= 0.0 || V.z <= 0.0) { s.w = 0.0; s.ev = EV_ABSORB; return s; }
    PrinEval e = principled_eval(m, comp, V, L);
    s.w = e.pdf > 0.0 ? e.fcos / e.pdf : 0.0;
    s.d = normalize(L.x * b1 + L.y * b2 + L.z * nf);
  } else if (m.type == GGX) {
    V3 b1, b2;
    onb(nf, b1, b2);
    V3 wo = -1.0 * d_in;
    V3 V = {dot(wo, b1), dot(wo, b2), dot(wo, nf)};
    V3 M = sample_vndf_local(V, m.rough, U.u[1], U.u[2]);
    double vm = dot(V, M);
    V3 L = (2.0 * vm) * M - V;
    s.ev = EV_GGX;
    if (L.z <= 0.0 || V.z <= 0.0) { s.w = 0.0; s.ev = EV_ABSORB; return s; }
    double f0 = m.rgb[comp];
    double F = f0 + (1.0 - f0) * std::pow(1.0 - std::max(0.0, vm), 5.0);
    s.w = F * smith_g1(L, m.rough);
    s.d = normalize(L.x * b1 + L.y * b2 + L.z * nf);
  }
  return s;
}

// ------------------------------------------------------------------ cache
// Round a double to IEEE binary16 with round-to-nearest-even and back.
double round_fp16(double x) {
  if (!(x == x)) return x;
  double ax = std::fabs(x);
  if (ax >= 65520.0) return std::copysign(INFINITY, x);
  int e;
  std::frexp(ax, &e);              // ax = f * 2^e, f in [0.5,1)
  int exp2 = e - 1;                // ax in [2^exp2, 2^(exp2+1))
  if (exp2 < -14) exp2 = -14;      // subnormal spacing 2^-24
  double ulp = std::ldexp(1.0, exp2 - 10);
  double q = ax / ulp;             // exact (power-of-two scaling)
  double fl = std::floor(q);
  double rem = q - fl;
  if (rem > 0.5 || (rem == 0.5 && std::fmod(fl, 2.0) != 0.0)) fl += 1.0;
  return std::copysign(fl * ulp, x);
}

// Octahedral map of a unit direction onto [-1,1]^2 and back.
void oct_encode(V3 w, double &u, double &v) {
  double s = std::fabs(w.x) + std::fabs(w.y) + std::fabs(w.z);
  double px = w.x / s, py = w.y / s;
  if (w.z < 0) {
    double sx = px >= 0 ? 1.0 : -1.0, sy = py >= 0 ? 1.0 : -1.0;
    double nx = (1.0 - std::fabs(py)) * sx, ny = (1.0 - std::fabs(px)) * sy;
    px = nx; py = ny;
  }
  u = px; v = py;
}

V3 oct_decode(double u, double v) {
  double z = 1.0 - std::fabs(u) - std::fabs(v);
  double x = u, y = v;
  if (z < 0) {
    double sx = x >= 0 ? 1.0 : -1.0, sy = y >= 0 ? 1.0 : -1.0;
    double nx = (1.0 - std::fabs(y)) * sx, ny = (1.0 - std::fabs(x)) * sy;
    x = nx; y = ny;
  }
  return normalize(V3{x, y, z});
}

int oct_bin(V3 w, int bins) {
  double u, v;
  oct_encode(w, u, v);
  int bu = (int)std::floor((u + 1.0) * 0.5 * bins);
  int bv = (int)std::floor((v + 1.0) * 0.5 * bins);
  bu = std::min(std::max(bu, 0), bins - 1);
  bv = std::min(std::max(bv, 0), bins - 1);
  return bv * bins + bu;
}

struct CacheParams { int res, bins, spb, max_bounces; uint64_t seed; };

struct Cache {
  const Scene *S;
  CacheParams P;
  V3 lo, hi;
  std::mutex mu;
  std::unordered_map<uint64_t, double> memo;   // key: comp | cell | bin
};

int cell_of(const Cache &C, V3 x) {
  int idx[3];
  for (int a = 0; a < 3; ++a) {
    double lo = comp_of(C.lo, a), hi = comp_of(C.hi, a);
    int i = (int)std::floor((comp_of(x, a) - lo) / (hi - lo) * C.P.res);
    idx[a] = std::min(std::max(i, 0), C.P.res - 1);
  }
  return (idx[2] * C.P.res + idx[1]) * C.P.res + idx[0];
}

// ------------------------------------------------------------------ paths
struct TraceCtx {
  const Scene *S;
  const Cache *cache;     // null: no cache
  int max_bounces;
  int cache_depth;
  double tmin;
  bool nee = false;       // next-event estimation to the emitter triangles, MIS-weighted
};

// f cos and sampling pdf (solid angle, of the lobe sample_bsdf draws) of the
// non-delta lobe of m for the direction wl leaving the surface; d_in: the
// incoming travel direction, cosines against the normal facing it. GGX:
// f cos = F D G1(V) G1(L) / (4 V.z), pdf = G1(V) D / (4 V.z), so that
// f cos / pdf is the sampling weight F G1(L).
struct Eval { double fcos, pdf; };
Eval eval_bsdf(const Material &m, int comp, V3 d_in, V3 ng, V3 wl) {
  V3 nf = dot(d_in, ng) < 0 ? ng : -1.0 * ng;
  double c = dot(wl, nf);
  if (c <= 0.0) return {0.0, 0.0};
  if (m.type == LAMBERT) return {m.rgb[comp] * c / M_PI, c / M_PI};
  if (m.type == PRINCIPLED) {
    V3 b1, b2;
    onb(nf, b1, b2);
    V3 wo = -1.0 * d_in;
    PrinEval e = principled_eval(m, comp, {dot(wo, b1), dot(wo, b2), dot(wo, nf)},
                                 {dot(wl, b1), dot(wl, b2), c});
    return {e.fcos, e.pdf};
  }
  if (m.type != GGX) return {0.0, 0.0};
  V3 b1, b2;
  onb(nf, b1, b2);
  V3 wo = -1.0 * d_in;
  V3 V = {dot(wo, b1), dot(wo, b2), dot(wo, nf)};
  V3 L = {dot(wl, b1), dot(wl, b2), c};
  if (V.z <= 0.0) return {0.0, 0.0};
  V3 H = normalize(V + L);
  double a2 = m.rough * m.rough;
  double k = H.z * H.z * (a2 - 1.0) + 1.0;
  double D = a2 / (M_PI * k * k);
  double f0 = m.rgb[comp];
  double F = f0 + (1.0 - f0) * std::pow(1.0 - std::max(0.0, dot(V, H)), 5.0);
  double pdf = smith_g1(V, m.rough) * D / (4.0 * V.z);
  return {pdf * F * smith_g1(L, m.rough), pdf};
}

// Next-event estimate at the non-delta vertex x (material m, primitive gid,
// reached along d_in): an emitter triangle chosen with probability
// proportional to area (u0), a point uniform on it (u1, u2), the
// unoccluded one-sided emission times f cos over the light pdf
// dist^2 / (cos_y A_total), weighted by the power heuristic against the
// lobe's pdf. The light index and visibility enter the signature.
double next_event(const TraceCtx &X, const Material &m, int comp, V3 x, V3 d_in, V3 ng, int gid,
                  const double u[3], uint64_t &sig) {
  const Scene &S = *X.S;
  int n = (int)S.lights.size();
  int i = (int)(std::upper_bound(S.light_cdf.begin(), S.light_cdf.end(), u[0] * S.light_area) -
                S.light_cdf.begin());
  i = std::min(i, n - 1);
  const Light &l = S.lights[i];
  double su = std::sqrt(u[1]);
  V3 y = (1.0 - su) * l.v0 + (su * (1.0 - u[2])) * l.v1 + (su * u[2]) * l.v2;
  V3 om = y - x;
  double dist = std::sqrt(dot(om, om));
  om = (1.0 / dist) * om;
  double cos_y = -dot(om, l.n);
  Eval e = eval_bsdf(m, comp, d_in, ng, om);
  bool vis = false;
  double c = 0.0;
  if (cos_y > 0.0 && e.fcos > 0.0) {
    int excl = gid >= S.n_sph ? gid : -1;
    Hit h = closest_hit(S, x, om, X.tmin, excl, false);
    vis = !(h.gid >= 0 && h.t < dist * (1.0 - 1e-4));
    if (vis) {
      double pl = dist * dist / (cos_y * S.light_area);
      double wl = pl * pl / (pl * pl + e.pdf * e.pdf);
      c = S.mats[l.mat].emit[comp] * e.fcos * wl / pl;
    }
  }
  sig_add(sig, 0x60000000u | (vis ? 0x800000u : 0u) | (uint32_t)i);
  return c;
}

double cache_lookup(Cache &C, int comp, int cell, int bin);

// Incoherent radiance from the interaction at x (index b), reached along
// d_in on primitive gid. Emitters add their one-sided emission and stop;
// other surfaces sample one lobe while b < max_bounces; escaped rays add the
// environment; a non-delta lobe at tail depth >= cache_depth returns the
// cached radiance instead of tracing (cache on). bP: index of the image point.
double radiance_tail(const TraceCtx &X, V3 x, V3 d_in, int gid, int b, int bP, int comp,
                     uint64_t seed, uint32_t key_a, uint32_t key_b, uint32_t stream_word,
                     uint64_t &sig, int &kind, Cache *cache_rw, int *n_hits, int *cell_out = nullptr,
                     int *bin_out = nullptr) {
  const Scene &S = *X.S;
  double L = 0.0, beta = 1.0;
  double eta = 1.0;
  const bool nee = X.nee && !S.lights.empty();
  double prev_pdf = 0.0, prev_t = 0.0;   // lobe pdf and length of the segment that led here (0: no MIS)
  for (;;) {
    const Material &m = S.mats[S.prim_mat[gid]];
    V3 ng = geom_normal(S, gid, x);
    if (m.type == EMITTER) {
      sig_add(sig, EV_EMIT);
      double cos_y = -dot(d_in, ng);
      if (cos_y > 0) {
        double wb = 1.0;   // power-heuristic weight of a lobe sample that next-event estimation also covers
        if (nee && prev_pdf > 0.0 && gid >= S.n_sph) {
          double pl = prev_t * prev_t / (cos_y * S.light_area);
          wb = prev_pdf * prev_pdf / (prev_pdf * prev_pdf + pl * pl);
        }
        L += beta * m.emit[comp] * wb;
      }
      kind = K_EMITTER;
      return L;
    }
    if (b >= X.max_bounces) { kind = K_MAXB_TAIL; return L; }
    uint32_t ctr[4] = {key_a, key_b, (uint32_t)b << 8, stream_word};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    philox4x32_10(ctr, key, w);
    Uniforms U;
    for (int i = 0; i < 4; ++i) U.u[i] = u01(w[i]);
    Sampled s = sample_bsdf(m, comp, d_in, ng, U, eta);
    sig_add(sig, (uint32_t)s.ev);
    const bool cache_here = X.cache && !s.delta && (b - bP + 1) >= X.cache_depth;
    const bool nee_here = nee && !s.delta && !cache_here;
    if (nee_here) {
      uint32_t c1[4] = {key_a, key_b, ((uint32_t)b << 8) | 1u, stream_word};
      uint32_t w1[4];
      philox4x32_10(c1, key, w1);
      double un[3] = {u01(w1[0]), u01(w1[1]), u01(w1[2])};
      L += beta * next_event(X, m, comp, x, d_in, ng, gid, un, sig);
    }
    if (s.w == 0.0) { kind = K_ABSORBED; return L; }
    prev_pdf = nee_here ? eval_bsdf(m, comp, d_in, ng, s.d).pdf : 0.0;
    beta *= s.w;
    if (s.ev == EV_DIEL_REFR) eta = s.eta_t;
    if (cache_here) {
      int cell = cell_of(*X.cache, x), bin = oct_bin(s.d, X.cache->P.bins);
      if (cell_out) *cell_out = cell;
      if (bin_out) *bin_out = bin;
      sig_add(sig, 0x40000000u | (uint32_t)cell);
      sig_add(sig, 0x50000000u | (uint32_t)bin);
      L += beta * cache_lookup(*cache_rw, comp, cell, bin);
      kind = K_CACHE;
      return L;
    }
    int excl = gid >= S.n_sph ? gid : -1;
    Hit h = closest_hit(S, x, s.d, X.tmin, excl, false);
    if (h.gid < 0) { L += beta * S.env[comp]; kind = K_ENV; sig_add(sig, 0xFFFFFFFEu); return L; }
    b += 1;
    if (n_hits) ++*n_hits;
    sig_add(sig, (uint32_t)h.gid + 1u);
    x = x + h.t * s.d;
    d_in = s.d;
    gid = h.gid;
    prev_t = h.t;
  }
}

// One cache entry: the mean over spb paths of the radiance seen from a point
// uniform in the cell, looking along a direction uniform in the bin's
// octahedral square, traced without the cache; stored as binary16 (RNE).
double cache_entry_fp64(const Cache &C, int comp, int cell, int bin) {
  const Scene &S = *C.S;
  int res = C.P.res, bins = C.P.bins;
  int ix = cell % res, iy = (cell / res) % res, iz = cell / (res * res);
  int bu = bin % bins, bv = bin / bins;
  TraceCtx X{&S, nullptr, C.P.max_bounces, 1, 1e-7};
  double sum = 0.0;
  uint32_t stream_word = ((uint32_t)comp << 16) | STREAM_CACHE;
  uint32_t key[2] = {(uint32_t)C.P.seed, (uint32_t)(C.P.seed >> 32)};
  for (int j = 0; j < C.P.spb; ++j) {
    uint32_t ka = (uint32_t)cell, kb = ((uint32_t)bin << 16) | (uint32_t)j;
    uint32_t c0[4] = {ka, kb, 0u, stream_word}, c1[4] = {ka, kb, 1u, stream_word};
    uint32_t w0[4], w1[4];
    philox4x32_10(c0, key, w0);
    philox4x32_10(c1, key, w1);
    V3 ext = C.hi - C.lo;
    V3 x = {C.lo.x + (ix + u01(w0[0])) / res * ext.x, C.lo.y + (iy + u01(w0[1])) / res * ext.y,
            C.lo.z + (iz + u01(w0[2])) / res * ext.z};
    double pu = -1.0 + 2.0 * (bu + u01(w0[3])) / bins;
    double pv = -1.0 + 2.0 * (bv + u01(w1[0])) / bins;
    V3 d = oct_decode(pu, pv);
    Hit h = closest_hit(S, x, d, 1e-7, -1, false);
    if (h.gid < 0) { sum += S.env[comp]; continue; }
    uint64_t sig = 0;
    int kind = 0;
    sum += radiance_tail(X, x + h.t * d, d, h.gid, 1, 1, comp, C.P.seed, ka, kb, stream_word,
                         sig, kind, nullptr, nullptr);
  }
  return sum / C.P.spb;
}

double cache_lookup(Cache &C, int comp, int cell, int bin) {
  uint64_t key = ((uint64_t)comp << 56) | ((uint64_t)cell << 16) | (uint64_t)bin;
  {
    std::lock_guard<std::mutex> g(C.mu);
    auto it = C.memo.find(key);
    if (it != C.memo.end()) return it->second;
  }
  double v = round_fp16(cache_entry_fp64(C, comp, cell, bin));
  std::lock_guard<std::mutex> g(C.mu);
  C.memo[key] = v;
  return v;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

struct OScene {
  const float *tri; int32_t n_tri; const uint32_t *tri_mat;
  const float *sph; int32_t n_sph; const uint32_t *sph_mat;
  int32_t n_mat; const uint32_t *mat_type; const float *mat_rgb; const float *mat_rough;
  const float *mat_ior; const float *mat_emit; const float *env;
  const float *mat_pbr;     // [n_mat][4] metallic, specular, clearcoat, clearcoat gloss (nullable)
  const float *pts;         // [n_pts][6] point emitters: position xyz, amplitude per component (nullable)
  int32_t n_pts;
};

struct OJob {
  int32_t width, height; double pitch;
  int32_t n_ch; double lambda[3]; int32_t comp[3];
  int32_t spp, max_bounces, T;
  uint64_t seed;
  int32_t random_phase, use_cache, cache_depth;
  int32_t crop[4];
  int32_t spp_begin, spp_end;
  double holo_from_world[12];
  int32_t grf_w, grf_h;
  const double *grf;        // complex128 [grf_h][grf_w][T] interleaved re, im
  int32_t nee;              // next-event estimation with MIS in the tail
  int32_t weight_mode;      // 0: W = r / p(v) (reading R); 1: W = 1 (Eq. 5 as printed, reading P)
};

struct ORecord {           // one per (channel, pixel, sample) path
  uint64_t sig;
  int32_t kind, bP, first_gid, n_hits;
  double ell, r, A, W, amp, qx, qy, rev;
  int32_t cache_cell, cache_bin;   // radiance-cache entry used (-1: none)
};

void *oracle_scene_create(const OScene *d) {
  Scene *S = new Scene();
  S->n_sph = d->n_sph; S->n_tri = d->n_tri;
  for (int i = 0; i < d->n_sph; ++i) {
    S->sc.push_back({d->sph[4 * i], d->sph[4 * i + 1], d->sph[4 * i + 2]});
    S->sr.push_back(d->sph[4 * i + 3]);
    S->prim_mat.push_back((int)d->sph_mat[i]);
  }
  for (int i = 0; i < d->n_tri; ++i) {
    for (int k = 0; k < 3; ++k)
      S->tv.push_back({d->tri[9 * i + 3 * k], d->tri[9 * i + 3 * k + 1], d->tri[9 * i + 3 * k + 2]});
    S->prim_mat.push_back((int)d->tri_mat[i]);
  }
  for (int i = 0; i < d->n_mat; ++i) {
    Material m;
    m.type = (int)d->mat_type[i];
    for (int c = 0; c < 3; ++c) { m.rgb[c] = d->mat_rgb[3 * i + c]; m.emit[c] = d->mat_emit[3 * i + c]; }
    m.rough = d->mat_rough[i]; m.ior = d->mat_ior[i];
    const float *pb = d->mat_pbr ? d->mat_pbr + 4 * i : nullptr;
    m.metallic = pb ? pb[0] : 0.0; m.specular = pb ? pb[1] : 0.5;
    m.clearcoat = pb ? pb[2] : 0.0; m.clearcoat_gloss = pb ? pb[3] : 1.0;
    S->mats.push_back(m);
  }
  for (int c = 0; c < 3; ++c) S->env[c] = d->env[c];
  for (int i = 0; i < d->n_pts; ++i) {
    const float *p = d->pts + 6 * i;
    S->pt_pos.push_back({p[0], p[1], p[2]});
    S->pt_amp.push_back({p[3], p[4], p[5]});
  }
  for (int i = 0; i < S->n_tri; ++i) {
    int mi = S->prim_mat[S->n_sph + i];
    if (S->mats[mi].type != EMITTER) continue;
    Light l;
    l.v0 = S->tv[3 * i]; l.v1 = S->tv[3 * i + 1]; l.v2 = S->tv[3 * i + 2];
    V3 cr = cross(l.v1 - l.v0, l.v2 - l.v0);
    double a2 = std::sqrt(dot(cr, cr));
    if (!(a2 > 0.0)) continue;
    l.n = (1.0 / a2) * cr;
    l.area = 0.5 * a2;
    l.mat = mi;
    S->light_area += l.area;
    S->lights.push_back(l);
    S->light_cdf.push_back(S->light_area);
  }
  int n = S->n_sph + S->n_tri;
  if (n > 0) {
    std::vector<Box> pb(n);
    std::vector<V3> pc(n);
    for (int g = 0; g < n; ++g) { pb[g] = prim_box(*S, g); pc[g] = 0.5 * (pb[g].lo + pb[g].hi); }
    S->order.resize(n);
    for (int g = 0; g < n; ++g) S->order[g] = g;
    build_node(*S, pb, pc, 0, n);
    S->bounds = pb[0];
    for (int g = 1; g < n; ++g) S->bounds = merge(S->bounds, pb[g]);
  } else {
    S->bounds = {{0, 0, 0}, {0, 0, 0}};
  }
  return S;
}

void oracle_scene_destroy(void *s) { delete (Scene *)s; }

void *oracle_cache_create(void *scene, int32_t res, int32_t bins, int32_t spb,
                          int32_t max_bounces, uint64_t seed) {
  Scene *S = (Scene *)scene;
  Cache *C = new Cache();
  C->S = S;
  C->P = {res, bins, spb, max_bounces, seed};
  // grid: the scene bounds inflated by 1e-3 of the largest extent
  V3 e = S->bounds.hi - S->bounds.lo;
  double pad = 1e-3 * std::max({e.x, e.y, e.z});
  C->lo = S->bounds.lo - V3{pad, pad, pad};
  C->hi = S->bounds.hi + V3{pad, pad, pad};
  return C;
}

void oracle_cache_destroy(void *c) { delete (Cache *)c; }

double oracle_cache_entry(void *c, int32_t comp, int32_t cell, int32_t bin, int32_t rounded) {
  Cache *C = (Cache *)c;
  return rounded ? cache_lookup(*C, comp, cell, bin) : cache_entry_fp64(*C, comp, cell, bin);
}

// Many entries at once (binary16-rounded values), in parallel.
void oracle_cache_entries(void *c, int64_t n, const int32_t *comp, const int32_t *cell,
                          const int32_t *bin, double *out, int32_t n_threads) {
  Cache *C = (Cache *)c;
  int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 64) num_threads(nt)
  for (int64_t i = 0; i < n; ++i) out[i] = cache_lookup(*C, comp[i], cell[i], bin[i]);
}

void oracle_cache_bounds(void *c, double *lo_hi) {
  Cache *C = (Cache *)c;
  lo_hi[0] = C->lo.x; lo_hi[1] = C->lo.y; lo_hi[2] = C->lo.z;
  lo_hi[3] = C->hi.x; lo_hi[4] = C->hi.y; lo_hi[5] = C->hi.z;
}

// Random spectral phases of Eq. 4: xi_t(jx, jy) = 2 pi u for DFT bins inside
// the passband f_x^2 + f_y^2 <= (1/2d)^2 (sin(theta_max)/lambda = 1/(2d), so
// the band is the disc inscribed in the sampled spectrum, independent of
// lambda); out-of-band bins get mask 0. Frames [t0, t0+nt); output [nt][gh][gw].
void oracle_grf_phases(int32_t gw, int32_t gh, int32_t t0, int32_t nt, uint64_t seed,
                       double *xi, uint8_t *mask) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int t = t0; t < t0 + nt; ++t)
    for (int jy = 0; jy < gh; ++jy)
      for (int jx = 0; jx < gw; ++jx) {
        int64_t sx = jx < (gw + 1) / 2 ? jx : jx - gw;   // signed frequency index
        int64_t sy = jy < (gh + 1) / 2 ? jy : jy - gh;
        // (sx/gw)^2 + (sy/gh)^2 <= 1/4, in exact integers
        bool in = 4 * (sx * sx * (int64_t)gh * gh + sy * sy * (int64_t)gw * gw) <=
                  (int64_t)gw * gw * (int64_t)gh * gh;
        size_t o = ((size_t)(t - t0) * gh + jy) * gw + jx;
        mask[o] = in ? 1 : 0;
        if (in) {
          uint32_t ctr[4] = {(uint32_t)jx, (uint32_t)jy, (uint32_t)t, STREAM_GRF};
          uint32_t w[4];
          philox4x32_10(ctr, key, w);
          xi[o] = 2.0 * M_PI * u01(w[0]);
        } else {
          xi[o] = 0.0;
        }
      }
}

void oracle_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out) {
  philox4x32_10(ctr, key, out);
}

// Test hooks for the pieces of the estimator.
void oracle_closest_hit(void *scene, const double *o, const double *d, double tmin,
                        int32_t exclude, int32_t brute, double *t_out, int32_t *gid_out) {
  Scene *S = (Scene *)scene;
  Hit h = closest_hit(*S, {o[0], o[1], o[2]}, {d[0], d[1], d[2]}, tmin, exclude, brute != 0);
  *t_out = h.t; *gid_out = h.gid;
}

double oracle_fresnel(double cos_i, double eta_i, double eta_t) {
  double ct;
  return fresnel_dielectric(cos_i, eta_i, eta_t, ct);
}

void oracle_sample_lambert(const double *n, double u1, double u2, double *out) {
  V3 d = sample_lambert({n[0], n[1], n[2]}, u1, u2);
  out[0] = d.x; out[1] = d.y; out[2] = d.z;
}

void oracle_sample_vndf(const double *V, double alpha, double u1, double u2, double *out) {
  V3 m = sample_vndf_local({V[0], V[1], V[2]}, alpha, u1, u2);
  out[0] = m.x; out[1] = m.y; out[2] = m.z;
}

double oracle_smith_g1(const double *w, double alpha) { return smith_g1({w[0], w[1], w[2]}, alpha); }

// Principled lobes of one colour component: p = (base, roughness, metallic,
// specular, clearcoat, clearcoat gloss); V, L local (z = facing normal).
static Material principled_of(const double *p) {
  Material m{};
  m.type = PRINCIPLED;
  m.rgb[0] = m.rgb[1] = m.rgb[2] = p[0];
  m.rough = p[1]; m.metallic = p[2]; m.specular = p[3]; m.clearcoat = p[4]; m.clearcoat_gloss = p[5];
  return m;
}

void oracle_principled_eval(const double *p, const double *V, const double *L, double *out) {
  PrinEval e = principled_eval(principled_of(p), 0, {V[0], V[1], V[2]}, {L[0], L[1], L[2]});
  out[0] = e.fcos; out[1] = e.pdf;
}

// Sampled local direction, its weight f cos / pdf (0 below the horizon) and lobe.
void oracle_principled_sample(const double *p, const double *V, const double *u, double *L_out, double *w,
                              int32_t *lobe) {
  Material m = principled_of(p);
  V3 v = {V[0], V[1], V[2]};
  int lb;
  V3 L = principled_sample(m, v, u[0], u[1], u[2], lb);
  *lobe = lb;
  L_out[0] = L.x; L_out[1] = L.y; L_out[2] = L.z;
  PrinEval e = principled_eval(m, 0, v, L);
  *w = (L.z > 0.0 && e.pdf > 0.0) ? e.fcos / e.pdf : 0.0;
}

void oracle_oct(const double *w, int32_t bins, double *uv, int32_t *bin) {
  double u, v;
  oct_encode({w[0], w[1], w[2]}, u, v);
  uv[0] = u; uv[1] = v;
  *bin = oct_bin({w[0], w[1], w[2]}, bins);
}

void oracle_oct_decode(double u, double v, double *w) {
  V3 d = oct_decode(u, v);
  w[0] = d.x; w[1] = d.y; w[2] = d.z;
}

double oracle_round_fp16(double x) { return round_fp16(x); }

// Phase of frame t at the hologram-space point (qx, qy): bilinear
// interpolation of the complex field r_t with periodic wrap, then its
// argument as a unit phasor (phase 0 if the interpolated value is exactly
// 0). Texel (i, j) sits on the centre of recording-plane pixel (i, j).
static std::complex<double> grf_phasor(const OJob &J, int t, double qx, double qy) {
  double u = qx / J.pitch + J.width * 0.5 - 0.5;
  double v = qy / J.pitch + J.height * 0.5 - 0.5;
  double fu = std::floor(u), fv = std::floor(v);
  double ax = u - fu, ay = v - fv;
  int64_t i0 = (int64_t)fu, j0 = (int64_t)fv;
  auto texel = [&](int64_t i, int64_t j) {
    int64_t ii = ((i % J.grf_w) + J.grf_w) % J.grf_w;
    int64_t jj = ((j % J.grf_h) + J.grf_h) % J.grf_h;
    const double *p = J.grf + 2 * (((size_t)jj * J.grf_w + ii) * J.T + t);
    return std::complex<double>(p[0], p[1]);
  };
  std::complex<double> r = (1 - ax) * (1 - ay) * texel(i0, j0) + ax * (1 - ay) * texel(i0 + 1, j0) +
                           (1 - ax) * ay * texel(i0, j0 + 1) + ax * ay * texel(i0 + 1, j0 + 1);
  double m = std::abs(r);
  return m > 0 ? r / m : std::complex<double>(1.0, 0.0);
}

// Inverse of the affine map x -> A x + b given row-major [A | b].
static void affine_inverse(const double *Tm, double *Ti) {
  double a = Tm[0], b = Tm[1], c = Tm[2], d = Tm[4], e = Tm[5], f = Tm[6], g = Tm[8], h = Tm[9],
         i = Tm[10];
  double A = e * i - f * h, B = -(d * i - f * g), C = d * h - e * g;
  double det = a * A + b * B + c * C;
  double inv[9] = {A / det, -(b * i - c * h) / det, (b * f - c * e) / det,
                   B / det, (a * i - c * g) / det, -(a * f - c * d) / det,
                   C / det, -(a * h - b * g) / det, (a * e - b * d) / det};
  for (int r = 0; r < 3; ++r) {
    for (int k = 0; k < 3; ++k) Ti[4 * r + k] = inv[3 * r + k];
    Ti[4 * r + 3] = -(inv[3 * r] * Tm[3] + inv[3 * r + 1] * Tm[7] + inv[3 * r + 2] * Tm[11]);
  }
}

static V3 apply_affine(const double *M, V3 x) {
  return {M[0] * x.x + M[1] * x.y + M[2] * x.z + M[3], M[4] * x.x + M[5] * x.y + M[6] * x.z + M[7],
          M[8] * x.x + M[9] * x.y + M[10] * x.z + M[11]};
}
static V3 apply_linear(const double *M, V3 x) {
  return {M[0] * x.x + M[1] * x.y + M[2] * x.z, M[4] * x.x + M[5] * x.y + M[6] * x.z,
          M[8] * x.x + M[9] * x.y + M[10] * x.z};
}

void oracle_grf_lookup(const OJob *J, int32_t t, double qx, double qy, double *out) {
  std::complex<double> p = grf_phasor(*J, t, qx, qy);
  out[0] = p.real(); out[1] = p.imag();
}

// Point emitter (a test primitive outside the paper's scenes; Eq. 2 for a
// source concentrated at one point with isotropic amplitude a, so the
// obliquity factor is 1): pixel p of the recording plane receives
// a exp(i (k r + phi_t(Q))) / r, with Q = T y the emitter in hologram space
// and r = |Q - x_p|, when Q lies in front of the plane inside the recordable
// cone (the direction cosines of Q - x_p within the disc of radius
// lambda/2d, boundary included, as for the sampled directions) and no scene
// primitive lies on the world-space segment from T^-1 x_p to y. The term is
// exact (not sampled); a job adds it once, in the sample range that starts
// at sample 0. acc: the pixel's T frame sums.
static void add_point_emitters(const Scene &S, const OJob &J, const double *Tinv, V3 xp, int comp,
                               double k, double s, std::complex<double> *acc) {
  for (size_t e = 0; e < S.pt_pos.size(); ++e) {
    double a = comp_of(S.pt_amp[e], comp);
    if (a == 0.0) continue;
    V3 y = S.pt_pos[e];
    V3 Q = apply_affine(J.holo_from_world, y);
    V3 dq = Q - xp;
    double r = length(dq);
    if (!(dq.z > 0.0) || dq.x * dq.x + dq.y * dq.y > s * s * r * r) continue;
    V3 O = apply_affine(Tinv, xp);
    V3 seg = y - O;
    double dist = length(seg);
    Hit h = closest_hit(S, O, (1.0 / dist) * seg, 1e-7, -1, false);
    if (h.gid >= 0 && h.t < dist) continue;
    std::complex<double> base = (a / r) * std::exp(std::complex<double>(0.0, k * r));
    for (int t = 0; t < J.T; ++t)
      acc[t] += J.random_phase ? base * grf_phasor(J, t, Q.x, Q.y) : base;
  }
}

// Trace every (channel, pixel, sample) path of the crop and accumulate the T
// frames. field: complex128 [n_ch][T][crop_h][crop_w]; recs (nullable):
// [n_ch][crop_h][crop_w][spp_end - spp_begin]; recs_t (nullable): per-path
// complex128 contribution of every frame, [n_ch][crop_h][crop_w][n_s][T].
// Returns 0, or -1 for invalid input.
int32_t oracle_trace(void *scene, void *cache, const OJob *J, double *field, ORecord *recs,
                     double *recs_t, int32_t n_threads) {
  Scene *S = (Scene *)scene;
  Cache *C = (Cache *)cache;
  if (J->n_ch < 1 || J->n_ch > 3 || J->T < 1 || J->spp < 1 || J->grf == nullptr) return -1;
  int x0 = J->crop[0], y0 = J->crop[1], cw = J->crop[2], ch = J->crop[3];
  if (cw == 0 || ch == 0) { x0 = 0; y0 = 0; cw = J->width; ch = J->height; }
  int sb = J->spp_begin, se = J->spp_end;
  if (sb == 0 && se == 0) se = J->spp;
  int ns = se - sb;
  double Tinv[12];
  affine_inverse(J->holo_from_world, Tinv);
  const double d = J->pitch;
  TraceCtx X{S, (J->use_cache && C) ? C : nullptr, J->max_bounces, J->cache_depth, 1e-7};
  X.nee = J->nee != 0;
  std::memset(field, 0, sizeof(double) * 2 * (size_t)J->n_ch * J->T * cw * ch);
  int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
  for (int row = 0; row < J->n_ch * ch; ++row) {
    int c = row / ch, yy = row % ch;
    int comp = J->comp[c];
    double lam = J->lambda[c];
    double k = 2.0 * M_PI / lam;
    double s = lam / (2.0 * d);                     // sin(theta_max)
    int py = y0 + yy;
    std::vector<std::complex<double>> acc((size_t)J->T);
    for (int xx = 0; xx < cw; ++xx) {
      int px = x0 + xx;
      uint32_t pixel = (uint32_t)py * (uint32_t)J->width + (uint32_t)px;
      V3 xp = {((px + 0.5) - J->width * 0.5) * d, ((py + 0.5) - J->height * 0.5) * d, 0.0};
      std::fill(acc.begin(), acc.end(), std::complex<double>(0, 0));
      for (int si = 0; si < ns; ++si) {
        uint32_t smp = (uint32_t)(sb + si);
        ORecord R{};
        R.first_gid = -1;
        R.cache_cell = -1;
        R.cache_bin = -1;
        uint64_t sig = FNV_OFFSET;
        // s1: direction cosines uniform on the disc alpha^2 + beta^2 <= s^2
        Uniforms U0 = path_uniforms(J->seed, pixel, smp, 0, (uint32_t)comp);
        double rad = s * std::sqrt(U0.u[0]), ang = 2.0 * M_PI * U0.u[1];
        double al = rad * std::cos(ang), be = rad * std::sin(ang);
        V3 v = {al, be, std::sqrt(1.0 - al * al - be * be)};
        // s2: to world space through the inverse of T
        V3 O = apply_affine(Tinv, xp);
        V3 dw = normalize(apply_linear(Tinv, v));
        // s3-s4: coherent prefix through delta lobes, OPL = sum n_i L_i
        V3 o = O, dir = dw;
        double ell = 0.0, ncur = 1.0, beta_pre = 1.0;
        int b = 0, excl = -1, kind = K_NONE, gid = -1;
        bool found = false;
        for (;;) {
          Hit h = closest_hit(*S, o, dir, X.tmin, excl, false);
          if (h.gid < 0) { kind = K_ESCAPE_PREFIX; sig_add(sig, 0xFFFFFFFFu); break; }
          b += 1;
          if (b == 1) R.first_gid = h.gid;
          sig_add(sig, (uint32_t)h.gid + 1u);
          if (b > J->max_bounces) { kind = K_MAXB_PREFIX; break; }
          ell += ncur * h.t;
          V3 xh = o + h.t * dir;
          const Material &m = S->mats[S->prim_mat[h.gid]];
          if (m.type == MIRROR || m.type == DIELECTRIC) {
            Uniforms Ub = path_uniforms(J->seed, pixel, smp, (uint32_t)b, (uint32_t)comp);
            Sampled sm = sample_bsdf(m, comp, dir, geom_normal(*S, h.gid, xh), Ub, ncur);
            sig_add(sig, (uint32_t)sm.ev);
            beta_pre *= sm.w;
            if (sm.ev == EV_DIEL_REFR) ncur = sm.eta_t;
            o = xh; dir = sm.d;
            excl = h.gid >= S->n_sph ? h.gid : -1;
            continue;
          }
          found = true;
          gid = h.gid;
          o = xh;
          sig_add(sig, EV_IMAGE_POINT);
          break;
        }
        R.n_hits = b;
        if (found) {
          // s6-s7: virtual image point P' = O + d_OPL v, Q = T P', r = |Q - x_p|
          V3 Pp = O + ell * dw;
          V3 Q = apply_affine(J->holo_from_world, Pp);
          double r = length(Q - xp);
          // weight of Eq. 2 per unit solid angle divided by the disc density
          // (reading R); Eq. 5 as printed has no weight (reading P: W = 1)
          double pdf = v.z / (M_PI * s * s);
          double W = J->weight_mode == 1 ? 1.0 : r / pdf;
          // s5: incoherent amplitude from the image point
          int tk = 0, nh = 0;
          double Lhat = radiance_tail(X, o, dir, gid, b, b, comp, J->seed, pixel, smp,
                                      ((uint32_t)comp << 16) | STREAM_PATH, sig, tk, C, &nh,
                                      &R.cache_cell, &R.cache_bin);
          kind = tk;
          double A = std::sqrt(beta_pre * Lhat);
          double amp = A * W / J->spp;
          double rev = r / lam - std::floor(r / lam);
          R.bP = b; R.ell = ell; R.r = r; R.A = A; R.W = W; R.amp = amp;
          R.qx = Q.x; R.qy = Q.y; R.rev = rev; R.n_hits = b + nh;
          // s8-s9: every frame reuses the path; only phi_t depends on t
          std::complex<double> base = amp * std::exp(std::complex<double>(0.0, k * r));
          for (int t = 0; t < J->T; ++t) {
            std::complex<double> ph =
                J->random_phase ? grf_phasor(*J, t, Q.x, Q.y) : std::complex<double>(1.0, 0.0);
            std::complex<double> cval = base * ph;
            acc[t] += cval;
            if (recs_t) {
              size_t ri = ((((size_t)c * ch + yy) * cw + xx) * ns + si) * J->T + t;
              recs_t[2 * ri] = cval.real(); recs_t[2 * ri + 1] = cval.imag();
            }
          }
        } else if (recs_t) {
          for (int t = 0; t < J->T; ++t) {
            size_t ri = ((((size_t)c * ch + yy) * cw + xx) * ns + si) * J->T + t;
            recs_t[2 * ri] = 0.0; recs_t[2 * ri + 1] = 0.0;
          }
        }
        sig_add(sig, 0x100u | (uint32_t)kind);
        R.sig = sig; R.kind = kind;
        if (recs) recs[(((size_t)c * ch + yy) * cw + xx) * ns + si] = R;
      }
      if (sb == 0) add_point_emitters(*S, *J, Tinv, xp, comp, k, s, acc.data());
      for (int t = 0; t < J->T; ++t) {
        size_t o = (((size_t)c * J->T + t) * ch + yy) * cw + xx;
        field[2 * o] = acc[t].real(); field[2 * o + 1] = acc[t].imag();
      }
    }
  }
  return 0;
}

}  // extern "C"
