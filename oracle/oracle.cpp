// CPU oracle for the differentiable EWA surfel rasterizer of 3D Surface Splatting
// (3DSS).  TEST INFRASTRUCTURE: only the test suite, the smoke check and the
// benchmark's CPU-baseline leg load this library.  It shares no code, header,
// table or constant generator with the GPU renderer.
//
// Everything here is a plain, slow, brute-force reading of the paper in FP64:
// per pixel every surfel is intersected (no tiles, no bounding boxes, no
// batching), the covering fragments are sorted by the start of their depth
// interval and grouped with the interval-merging procedure of Alg. 1, each
// layer is Shepard-normalised (eq:shepard), given a coverage opacity
// (eq:alpha) and composited front to back (eq:compositing).  Forward shading
// is the split-sum model of eq:ibl (Sec. 3.4.2) over pre-filtered environment
// maps.  The scalar type is a template parameter: `double` gives values, `Dual`
// exact directional derivatives, and `Var` (a reverse-mode tape) the adjoint.
//
// The only FP32 code is `bin_f32`: the tile-binning decision (cull, depth key,
// tile rectangle), which the renderer takes in FP32, so the oracle takes it in
// FP32 too, following the fixed evaluation order documented with it.
//
// Parity pins: every function here is checked by the CPU test suite against
// closed forms, brute-force equivalences, dual-number JVPs and finite
// differences (tests/test_oracle_*.py).  The BRDF look-up table and the
// environment-map conventions are readings of silent points of the paper and
// are pinned only by internal properties ("parity unpinned" by the paper).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include <omp.h>

#include "ad.hpp"

namespace orc {
thread_local Tape* g_tape = nullptr;

static const double kPi = 3.14159265358979323846;

// ------------------------------------------------------------------ inputs
struct Cam {
  int W, H;
  double fx, fy, cx, cy;
  double R[9], t[3];
  double znear;
  double bg[3];
};
struct Opt {
  double r_cut, gamma, sigma_f;
  int k_max, shade, tile_w, tile_h;
  int mip;  // 0: centre-precomputed MIP filter (Sec. 3.3.2); 1: per-pixel Jacobian (Sec. 3.3.1)
  double t_min;  // transmittance early-out: the walk ends once T_{k+1} < t_min (0: off)
  int tonemap;   // 1: log-space + sRGB transfer of the image (eq:photo_loss, Sec. 3.7.1)
};
static Cam unpack_cam(const double* c) {
  Cam k;
  k.W = (int)c[0]; k.H = (int)c[1];
  k.fx = c[2]; k.fy = c[3]; k.cx = c[4]; k.cy = c[5];
  for (int i = 0; i < 9; ++i) k.R[i] = c[6 + i];
  for (int i = 0; i < 3; ++i) k.t[i] = c[15 + i];
  k.znear = c[18];
  for (int i = 0; i < 3; ++i) k.bg[i] = c[19 + i];
  return k;
}
static Opt unpack_opt(const double* o) {
  Opt p;
  p.r_cut = o[0]; p.gamma = o[1]; p.sigma_f = o[2];
  p.k_max = (int)o[3]; p.shade = (int)o[4]; p.tile_w = (int)o[5]; p.tile_h = (int)o[6];
  p.mip = (int)o[7];
  p.t_min = o[8];
  p.tonemap = (int)o[9];
  return p;
}

// Surfel parameters (Sec. 3.1): centre c, frame given as normal + tangent +
// two scales (t_u = s_u u_hat, t_v = s_v v_hat), albedo, roughness, metallic.
template <class S> struct Surf { S p[3], n[3], t[3], s[2], alb[3], rough, metal; };

// Per (surfel, view) quantities: rows T1, T2, T4 of the T-matrix (Sec. 3.1,
// App. A.1), depth interval, centre-precomputed MIP filter (Sec. 3.3.2) and
// the forward-shaded colour (Sec. 3.4).
template <class S> struct Rec {
  S T1[3], T2[3], T4[3];
  S zs, ze;
  S sinv[3];  // Sigma_mip^{-1}: uu, uv, vv
  S sig[3];   // Sigma_mip itself: uu, uv, vv
  S nf;
  S col[3];
  int rect[4] = {0, -1, 0, -1};  // FP32 binning pixel rectangle il, ih, jl, jh
};

// ------------------------------------------------------------ environment maps
// Equirectangular, z-up.  Texel (a, b) of an H x W map has direction
// (sin th cos ph, sin th sin ph, cos th) with th = pi (a + 1/2)/H,
// ph = 2 pi (b + 1/2)/W.  Flat layout of the map set: level 0 (= E),
// specular levels 1..5, then the 32 x 64 irradiance map.
struct MapDims {
  int h[7], w[7];
  size_t off[8];
  MapDims(int He, int We) {
    h[0] = He; w[0] = We;
    for (int l = 1; l <= 5; ++l) { h[l] = std::max(He >> l, 4); w[l] = std::max(We >> l, 8); }
    h[6] = 32; w[6] = 64;
    off[0] = 0;
    for (int l = 0; l < 7; ++l) off[l + 1] = off[l] + (size_t)h[l] * w[l] * 3;
  }
  size_t total() const { return off[7]; }
};

static void texel_dir(int a, int b, int H, int W, double d[3]) {
  double th = kPi * (a + 0.5) / H, ph = 2.0 * kPi * (b + 0.5) / W;
  d[0] = std::sin(th) * std::cos(ph);
  d[1] = std::sin(th) * std::sin(ph);
  d[2] = std::cos(th);
}
static double texel_solid_angle(int a, int H, int W) {
  return (2.0 * kPi / W) * (std::cos(kPi * a / H) - std::cos(kPi * (a + 1) / H));
}
// GGX normal distribution D(mu; alpha) = alpha^2 / (pi (mu^2 (alpha^2 - 1) + 1)^2)
static double ggx_D(double mu, double alpha) {
  double a2 = alpha * alpha;
  double t = mu * mu * (a2 - 1.0) + 1.0;
  return a2 / (kPi * t * t);
}
// Prefilter weight of input texel direction dt for output direction R at GGX
// roughness alpha (split-sum prefilter with n = v = R, eq:ibl).
static double spec_weight(const double R[3], const double dt[3], double dOmega, double alpha) {
  double rl = R[0] * dt[0] + R[1] * dt[1] + R[2] * dt[2];
  if (rl <= 0.0) return 0.0;
  double h[3] = {R[0] + dt[0], R[1] + dt[1], R[2] + dt[2]};
  double hn = std::sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
  double mu = (R[0] * h[0] + R[1] * h[1] + R[2] * h[2]) / hn;
  return ggx_D(mu, alpha) * rl * dOmega;
}

// Irr(d) = (1/pi) sum_t E_t max(0, d.d_t) dOmega_t;
// Spec_l(R) = sum_t E_t K_l(R,t) / sum_t K_l(R,t), alpha_l = (l/5)^2.
// Generic in the scalar type so that a dual-number E gives the JVP.
template <class S>
static void envmap_prefilter(const S* E, int He, int We, S* maps) {
  MapDims md(He, We);
  size_t nt = (size_t)He * We;
  std::vector<double> dirs(nt * 3), dom(nt);
  for (int a = 0; a < He; ++a)
    for (int b = 0; b < We; ++b) {
      texel_dir(a, b, He, We, &dirs[((size_t)a * We + b) * 3]);
      dom[(size_t)a * We + b] = texel_solid_angle(a, He, We);
    }
  for (size_t i = 0; i < nt * 3; ++i) maps[i] = E[i];
  // irradiance
  {
    int H = md.h[6], W = md.w[6];
#pragma omp parallel for schedule(dynamic)
    for (int o = 0; o < H * W; ++o) {
      double d[3];
      texel_dir(o / W, o % W, H, W, d);
      S acc[3] = {S(0.0), S(0.0), S(0.0)};
      for (size_t t = 0; t < nt; ++t) {
        double c = d[0] * dirs[3 * t] + d[1] * dirs[3 * t + 1] + d[2] * dirs[3 * t + 2];
        if (c <= 0.0) continue;
        double k = c * dom[t] / kPi;
        for (int ch = 0; ch < 3; ++ch) acc[ch] += E[3 * t + ch] * k;
      }
      for (int ch = 0; ch < 3; ++ch) maps[md.off[6] + 3 * (size_t)o + ch] = acc[ch];
    }
  }
  for (int l = 1; l <= 5; ++l) {
    int H = md.h[l], W = md.w[l];
    double alpha = (l / 5.0) * (l / 5.0);
#pragma omp parallel for schedule(dynamic)
    for (int o = 0; o < H * W; ++o) {
      double R[3];
      texel_dir(o / W, o % W, H, W, R);
      S acc[3] = {S(0.0), S(0.0), S(0.0)};
      double z = 0.0;
      for (size_t t = 0; t < nt; ++t) {
        double k = spec_weight(R, &dirs[3 * t], dom[t], alpha);
        if (k == 0.0) continue;
        z += k;
        for (int ch = 0; ch < 3; ++ch) acc[ch] += E[3 * t + ch] * k;
      }
      for (int ch = 0; ch < 3; ++ch) maps[md.off[l] + 3 * (size_t)o + ch] = acc[ch] / z;
    }
  }
}

// Adjoint of the (linear) prefilter: dE = dSpec_0 + sum_l P_l^T dSpec_l + D^T dIrr.
static void envmap_adjoint(const double* dmaps, int He, int We, double* dE) {
  MapDims md(He, We);
  size_t nt = (size_t)He * We;
  std::vector<double> dirs(nt * 3), dom(nt);
  for (int a = 0; a < He; ++a)
    for (int b = 0; b < We; ++b) {
      texel_dir(a, b, He, We, &dirs[((size_t)a * We + b) * 3]);
      dom[(size_t)a * We + b] = texel_solid_angle(a, He, We);
    }
  for (size_t i = 0; i < nt * 3; ++i) dE[i] = dmaps[i];
  // normalisers of each specular output texel
  std::vector<std::vector<double>> Z(6);
  for (int l = 1; l <= 5; ++l) {
    int H = md.h[l], W = md.w[l];
    double alpha = (l / 5.0) * (l / 5.0);
    Z[l].assign((size_t)H * W, 0.0);
#pragma omp parallel for schedule(dynamic)
    for (int o = 0; o < H * W; ++o) {
      double R[3];
      texel_dir(o / W, o % W, H, W, R);
      double z = 0.0;
      for (size_t t = 0; t < nt; ++t) z += spec_weight(R, &dirs[3 * t], dom[t], alpha);
      Z[l][o] = z;
    }
  }
#pragma omp parallel for schedule(dynamic)
  for (long t = 0; t < (long)nt; ++t) {
    double acc[3] = {0, 0, 0};
    const double* dt = &dirs[3 * t];
    {
      int H = md.h[6], W = md.w[6];
      for (int o = 0; o < H * W; ++o) {
        double d[3];
        texel_dir(o / W, o % W, H, W, d);
        double c = d[0] * dt[0] + d[1] * dt[1] + d[2] * dt[2];
        if (c <= 0.0) continue;
        double k = c * dom[t] / kPi;
        for (int ch = 0; ch < 3; ++ch) acc[ch] += dmaps[md.off[6] + 3 * (size_t)o + ch] * k;
      }
    }
    for (int l = 1; l <= 5; ++l) {
      int H = md.h[l], W = md.w[l];
      double alpha = (l / 5.0) * (l / 5.0);
      for (int o = 0; o < H * W; ++o) {
        double R[3];
        texel_dir(o / W, o % W, H, W, R);
        double k = spec_weight(R, dt, dom[t], alpha);
        if (k == 0.0) continue;
        k /= Z[l][o];
        for (int ch = 0; ch < 3; ++ch) acc[ch] += dmaps[md.off[l] + 3 * (size_t)o + ch] * k;
      }
    }
    for (int ch = 0; ch < 3; ++ch) dE[3 * t + ch] += acc[ch];
  }
}

// ------------------------------------------------------------ BRDF table
// Split-sum scale/bias (beta1, beta2) of eq:ibl, indexed by (n.w_o, r).
// Reading of the paper's silent point: GGX with alpha = r^2, separable Smith
// masking-shadowing, Schlick Fresnel, M Hammersley samples of the GGX
// half-vector distribution; vertex (i, j) sits at r = i/(n_r-1),
// n.v = max(j/(n_nv-1), 1e-3).  Layout [n_r][n_nv][2].
static double radical_inverse2(uint32_t k) {
  k = (k << 16) | (k >> 16);
  k = ((k & 0x55555555u) << 1) | ((k & 0xAAAAAAAAu) >> 1);
  k = ((k & 0x33333333u) << 2) | ((k & 0xCCCCCCCCu) >> 2);
  k = ((k & 0x0F0F0F0Fu) << 4) | ((k & 0xF0F0F0F0u) >> 4);
  k = ((k & 0x00FF00FFu) << 8) | ((k & 0xFF00FF00u) >> 8);
  return (double)k * (1.0 / 4294967296.0);
}
static void brdf_lut(int n_nv, int n_r, int M, double* out) {
  for (int i = 0; i < n_r; ++i) {
    double r = (double)i / (n_r - 1), alpha = r * r, a2 = alpha * alpha;
    for (int j = 0; j < n_nv; ++j) {
      double nv = std::max((double)j / (n_nv - 1), 1e-3);
      double v[3] = {std::sqrt(1.0 - nv * nv), 0.0, nv};
      double A = 0.0, B = 0.0;
      for (int k = 0; k < M; ++k) {
        double xi1 = (k + 0.5) / M, xi2 = radical_inverse2((uint32_t)k);
        double ct = std::sqrt((1.0 - xi1) / (1.0 + (a2 - 1.0) * xi1));
        double st = std::sqrt(std::max(0.0, 1.0 - ct * ct));
        double ph = 2.0 * kPi * xi2;
        double h[3] = {st * std::cos(ph), st * std::sin(ph), ct};
        double vh = v[0] * h[0] + v[1] * h[1] + v[2] * h[2];
        double lz = 2.0 * vh * h[2] - v[2];
        if (lz <= 0.0) continue;
        double g1v = 2.0 * nv / (nv + std::sqrt(a2 + (1.0 - a2) * nv * nv));
        double g1l = 2.0 * lz / (lz + std::sqrt(a2 + (1.0 - a2) * lz * lz));
        double gvis = g1v * g1l * vh / (h[2] * nv);
        double fc = std::pow(1.0 - vh, 5.0);
        A += (1.0 - fc) * gvis;
        B += fc * gvis;
      }
      out[((size_t)i * n_nv + j) * 2 + 0] = A / M;
      out[((size_t)i * n_nv + j) * 2 + 1] = B / M;
    }
  }
}

// ------------------------------------------------------------ map accessors
// Read-only view of the map set in the scalar type S.
struct MapsD {
  const double* m;
  double get(size_t i) const { return m[i]; }
};
struct MapsDual {
  const double* m;
  const double* dm;
  Dual get(size_t i) const { return Dual(m[i], dm ? dm[i] : 0.0); }
};
struct MapsVar {  // leaves created on first use; their tape ids are recorded
  const double* m;
  mutable std::unordered_map<size_t, Var> used;
  Var get(size_t i) const {
    auto it = used.find(i);
    if (it != used.end()) return it->second;
    Var v = Var::leaf(m[i]);
    used.emplace(i, v);
    return v;
  }
};
struct Lut {
  const double* t;
  int n_nv, n_r;
};

template <class S> static S clamp01(S x) {
  if (val(x) < 0.0) return S(0.0);
  if (val(x) > 1.0) return S(1.0);
  return x;
}

// Bilinear lat-long lookup of level `l` along direction d (wrap in phi, clamp in
// theta, texel centres at +1/2).
template <class S, class M>
static void latlong(const M& maps, const MapDims& md, int l, const S d[3], S out[3]) {
  using std::atan2; using std::sqrt; using std::floor;
  int H = md.h[l], W = md.w[l];
  S rho = sqrt(d[0] * d[0] + d[1] * d[1]);
  S th = atan2(rho, d[2]);
  S ph = atan2(d[1], d[0]);
  if (val(ph) < 0.0) ph = ph + 2.0 * kPi;
  S a = th * (H / kPi) - 0.5;
  S b = ph * (W / (2.0 * kPi)) - 0.5;
  double a0 = std::floor(val(a)), b0 = std::floor(val(b));
  S fa = a - a0, fb = b - b0;
  int ra = std::min(std::max((int)a0, 0), H - 1), rb = std::min(std::max((int)a0 + 1, 0), H - 1);
  int ca = (((int)b0 % W) + W) % W, cb = (ca + 1) % W;
  for (int ch = 0; ch < 3; ++ch) {
    S v00 = maps.get(md.off[l] + 3 * ((size_t)ra * W + ca) + ch);
    S v01 = maps.get(md.off[l] + 3 * ((size_t)ra * W + cb) + ch);
    S v10 = maps.get(md.off[l] + 3 * ((size_t)rb * W + ca) + ch);
    S v11 = maps.get(md.off[l] + 3 * ((size_t)rb * W + cb) + ch);
    out[ch] = (1.0 - fa) * ((1.0 - fb) * v00 + fb * v01) + fa * ((1.0 - fb) * v10 + fb * v11);
  }
}

template <class S>
static void lut_lookup(const Lut& L, S nv, S r, S out[2]) {
  S x = nv * (double)(L.n_nv - 1), y = r * (double)(L.n_r - 1);
  int j0 = std::min((int)std::floor(val(x)), L.n_nv - 2);
  int i0 = std::min((int)std::floor(val(y)), L.n_r - 2);
  S fx = x - (double)j0, fy = y - (double)i0;
  for (int c = 0; c < 2; ++c) {
    double t00 = L.t[((size_t)i0 * L.n_nv + j0) * 2 + c];
    double t01 = L.t[((size_t)i0 * L.n_nv + j0 + 1) * 2 + c];
    double t10 = L.t[((size_t)(i0 + 1) * L.n_nv + j0) * 2 + c];
    double t11 = L.t[((size_t)(i0 + 1) * L.n_nv + j0 + 1) * 2 + c];
    out[c] = (1.0 - fy) * ((1.0 - fx) * t00 + fx * t01) + fy * ((1.0 - fx) * t10 + fx * t11);
  }
}

// ------------------------------------------------------------ per (surfel, view)
// Centre-precomputed MIP filter (Sec. 3.3.2): Sigma_mip = I + sigma_f J J^T with
// J = M^{-1} the inverse of the screen Jacobian at the surfel centre, and the
// normalisation n_f = sqrt(|I| / |Sigma_mip|).  A function of the T rows only,
// so that it can also be differentiated with respect to T.
template <class S>
static void mip_filter(Rec<S>& r, double sigma_f) {
  using std::sqrt;
  // M = d(x,y)/d(u,v) at u = v = 0 (quotient rule on x = T1.(u,v,1)/T4.(u,v,1))
  S z2 = r.T4[2] * r.T4[2];
  S M11 = (r.T1[0] * r.T4[2] - r.T1[2] * r.T4[0]) / z2;
  S M12 = (r.T1[1] * r.T4[2] - r.T1[2] * r.T4[1]) / z2;
  S M21 = (r.T2[0] * r.T4[2] - r.T2[2] * r.T4[0]) / z2;
  S M22 = (r.T2[1] * r.T4[2] - r.T2[2] * r.T4[1]) / z2;
  S detM = M11 * M22 - M12 * M21;
  // J = M^{-1}
  S J11 = M22 / detM, J12 = -M12 / detM, J21 = -M21 / detM, J22 = M11 / detM;
  // Sigma_mip = I + sigma_f J J^T
  S s11 = 1.0 + sigma_f * (J11 * J11 + J12 * J12);
  S s12 = sigma_f * (J11 * J21 + J12 * J22);
  S s22 = 1.0 + sigma_f * (J21 * J21 + J22 * J22);
  S dets = s11 * s22 - s12 * s12;
  r.sig[0] = s11;
  r.sig[1] = s12;
  r.sig[2] = s22;
  r.sinv[0] = s22 / dets;
  r.sinv[1] = -s12 / dets;
  r.sinv[2] = s11 / dets;
  r.nf = sqrt(1.0 / dets);
}

// Sec. 3.1: frame, camera-space vectors, T = P S with the pixel-space pinhole
// projection, depth extent eps_z = r_cut sqrt(t'_uz^2 + t'_vz^2).
// Sec. 3.3.2: J = d(u,v)/d(x,y) at the surfel centre, Sigma_mip = I + sigma_f J J^T
// (eq:mip_cov), n_f = sqrt(|I| / |Sigma_mip|) (eq:mip_eval).
// Sec. 3.4.2: split-sum shading (eq:ibl) at the surfel centre for this view.
template <class S, class M>
static void preprocess(const Surf<S>& s, const Cam& cam, const Opt& o, const M& maps,
                       const MapDims* md, const Lut* lut, Rec<S>& r) {
  using std::sqrt;
  // frame: n_hat, u_hat (Gram-Schmidt of the tangent), v_hat = n_hat x u_hat
  S nn = sqrt(s.n[0] * s.n[0] + s.n[1] * s.n[1] + s.n[2] * s.n[2]);
  S nh[3] = {s.n[0] / nn, s.n[1] / nn, s.n[2] / nn};
  S d = s.t[0] * nh[0] + s.t[1] * nh[1] + s.t[2] * nh[2];
  S g[3] = {s.t[0] - d * nh[0], s.t[1] - d * nh[1], s.t[2] - d * nh[2]};
  S gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  S uh[3] = {g[0] / gn, g[1] / gn, g[2] / gn};
  S vh[3] = {nh[1] * uh[2] - nh[2] * uh[1], nh[2] * uh[0] - nh[0] * uh[2],
             nh[0] * uh[1] - nh[1] * uh[0]};
  S tu[3], tv[3];
  for (int i = 0; i < 3; ++i) { tu[i] = s.s[0] * uh[i]; tv[i] = s.s[1] * vh[i]; }
  // camera space
  S cp[3], tup[3], tvp[3];
  for (int i = 0; i < 3; ++i) {
    const double* R = &cam.R[3 * i];
    cp[i] = R[0] * s.p[0] + R[1] * s.p[1] + R[2] * s.p[2] + cam.t[i];
    tup[i] = R[0] * tu[0] + R[1] * tu[1] + R[2] * tu[2];
    tvp[i] = R[0] * tv[0] + R[1] * tv[1] + R[2] * tv[2];
  }
  // T = P S; P = [[fx,0,cx,0],[0,fy,cy,0],[.,.,.,.],[0,0,1,0]], S = [t'_u t'_v 0 c']
  r.T1[0] = cam.fx * tup[0] + cam.cx * tup[2];
  r.T1[1] = cam.fx * tvp[0] + cam.cx * tvp[2];
  r.T1[2] = cam.fx * cp[0] + cam.cx * cp[2];
  r.T2[0] = cam.fy * tup[1] + cam.cy * tup[2];
  r.T2[1] = cam.fy * tvp[1] + cam.cy * tvp[2];
  r.T2[2] = cam.fy * cp[1] + cam.cy * cp[2];
  r.T4[0] = tup[2];
  r.T4[1] = tvp[2];
  r.T4[2] = cp[2];
  S ez = o.r_cut * sqrt(tup[2] * tup[2] + tvp[2] * tvp[2]);
  r.zs = cp[2] - ez;
  r.ze = cp[2] + ez;
  mip_filter(r, o.sigma_f);
  // colour
  if (o.shade == 0) {
    for (int c = 0; c < 3; ++c) r.col[c] = s.alb[c];
    return;
  }
  if (o.shade == 2) {  // normal image: the world-space unit normal is the attribute
    for (int c = 0; c < 3; ++c) r.col[c] = nh[c];
    return;
  }
  // camera centre in world space: o = -R^T t
  double oc[3];
  for (int j = 0; j < 3; ++j)
    oc[j] = -(cam.R[0 + j] * cam.t[0] + cam.R[3 + j] * cam.t[1] + cam.R[6 + j] * cam.t[2]);
  S wv[3] = {oc[0] - s.p[0], oc[1] - s.p[1], oc[2] - s.p[2]};
  S wl = sqrt(wv[0] * wv[0] + wv[1] * wv[1] + wv[2] * wv[2]);
  S wo[3] = {wv[0] / wl, wv[1] / wl, wv[2] / wl};
  S m = s.metal;
  S F0[3], kd[3];
  for (int c = 0; c < 3; ++c) {
    F0[c] = 0.04 * (1.0 - m) + s.alb[c] * m;
    kd[c] = (1.0 - F0[c]) * (1.0 - m);
  }
  S Ld[3];
  latlong(maps, *md, 6, nh, Ld);
  S nv = nh[0] * wo[0] + nh[1] * wo[1] + nh[2] * wo[2];
  S rd[3] = {2.0 * nv * nh[0] - wo[0], 2.0 * nv * nh[1] - wo[1], 2.0 * nv * nh[2] - wo[2]};
  S rc = clamp01(s.rough);
  S lam = 5.0 * rc;
  int l0 = std::min((int)std::floor(val(lam)), 4);
  S tl = lam - (double)l0;
  S A[3], B[3];
  latlong(maps, *md, l0, rd, A);
  latlong(maps, *md, l0 + 1, rd, B);
  S beta[2];
  lut_lookup(*lut, clamp01(nv), rc, beta);
  for (int c = 0; c < 3; ++c) {
    S Ls = (1.0 - tl) * A[c] + tl * B[c];
    r.col[c] = kd[c] * s.alb[c] * Ld[c] + Ls * (F0[c] * beta[0] + beta[1]);
  }
}

// ------------------------------------------------------------ FP32 binning
// The tile-binning decision in FP32 with a fixed evaluation order (no
// contraction, IEEE division and square root, sums left to right).  Outputs:
// keep flag, z_start bits, inclusive tile rectangle, pixel rectangle.
struct BinOut {
  // stage reached: 0 culled (centre not beyond znear), 1 culled (degenerate
  // projection, det A = 0), 2 culled (acceptance ellipse not entirely beyond
  // znear), 3 empty pixel rectangle (off screen or between pixel centres),
  // 4 kept
  int stage;
  int keep;
  float zs;
  int tx0, ty0, tx1, ty1;  // inclusive tile rectangle (empty: keep = 0)
  int il, ih, jl, jh;      // inclusive pixel rectangle
};
template <class S> static void set_rect(Rec<S>& r, const BinOut& b) {
  r.rect[0] = b.il; r.rect[1] = b.ih; r.rect[2] = b.jl; r.rect[3] = b.jh;
}

static BinOut bin_f32(const float* const* P, int n, int i, const Cam& cd, const Opt& od) {
  BinOut b{0, 0, 0.f, 0, 0, -1, -1, 0, -1, 0, -1};
  const float nx = P[1][i], ny = P[1][n + i], nz = P[1][2 * n + i];
  const float tx = P[2][i], ty = P[2][n + i], tz = P[2][2 * n + i];
  const float su = P[3][i], sv = P[3][n + i];
  const float px = P[0][i], py = P[0][n + i], pz = P[0][2 * n + i];
  float R[9], t[3];
  for (int k = 0; k < 9; ++k) R[k] = (float)cd.R[k];
  for (int k = 0; k < 3; ++k) t[k] = (float)cd.t[k];
  const float fx = (float)cd.fx, fy = (float)cd.fy, cx = (float)cd.cx, cy = (float)cd.cy;
  const float znear = (float)cd.znear, rcut = (float)od.r_cut, sigma = (float)od.sigma_f;
  float nn = std::sqrt(nx * nx + ny * ny + nz * nz);
  float nhx = nx / nn, nhy = ny / nn, nhz = nz / nn;
  float d = tx * nhx + ty * nhy + tz * nhz;
  float gx = tx - d * nhx, gy = ty - d * nhy, gz = tz - d * nhz;
  float gn = std::sqrt(gx * gx + gy * gy + gz * gz);
  float ux = gx / gn, uy = gy / gn, uz = gz / gn;
  float vx = nhy * uz - nhz * uy, vy = nhz * ux - nhx * uz, vz = nhx * uy - nhy * ux;
  float tux = su * ux, tuy = su * uy, tuz = su * uz;
  float tvx = sv * vx, tvy = sv * vy, tvz = sv * vz;
  float cpx = R[0] * px + R[1] * py + R[2] * pz + t[0];
  float cpy = R[3] * px + R[4] * py + R[5] * pz + t[1];
  float cpz = R[6] * px + R[7] * py + R[8] * pz + t[2];
  float upx = R[0] * tux + R[1] * tuy + R[2] * tuz;
  float upy = R[3] * tux + R[4] * tuy + R[5] * tuz;
  float upz = R[6] * tux + R[7] * tuy + R[8] * tuz;
  float vpx = R[0] * tvx + R[1] * tvy + R[2] * tvz;
  float vpy = R[3] * tvx + R[4] * tvy + R[5] * tvz;
  float vpz = R[6] * tvx + R[7] * tvy + R[8] * tvz;
  float z = cpz;
  float ez = rcut * std::sqrt(upz * upz + vpz * vpz);
  b.zs = z - ez;
  if (!(z > znear)) return b;
  b.stage = 1;
  float mx = cpx / z, my = cpy / z;
  float x0 = fx * mx + cx, y0 = fy * my + cy;
  float M11 = (fx * (upx - mx * upz)) / z, M12 = (fx * (vpx - mx * vpz)) / z;
  float M21 = (fy * (upy - my * upz)) / z, M22 = (fy * (vpy - my * vpz)) / z;
  float g1 = upz / z, g2 = vpz / z;
  float dm = M11 * M22 - M12 * M21;
  float detA = dm * dm;
  if (!(detA > 0.f)) return b;
  b.stage = 2;
  float a = M11 * M11 + M21 * M21, bb = M11 * M12 + M21 * M22, c = M12 * M12 + M22 * M22;
  float S11 = detA + sigma * c, S12 = -(sigma * bb), S22 = detA + sigma * a;
  float Sg1 = S11 * g1 + S12 * g2, Sg2 = S12 * g1 + S22 * g2;
  float gSg = g1 * Sg1 + g2 * Sg2;
  float r2 = rcut * rcut;
  float kz = 1.f - znear / z;
  if (!(r2 * gSg < detA * (kz * kz))) return b;
  b.stage = 3;
  float den = detA - r2 * gSg;
  float SM1x = S11 * M11 + S12 * M12, SM1y = S12 * M11 + S22 * M12;
  float M1SM1 = M11 * SM1x + M12 * SM1y, M1Sg = M11 * Sg1 + M12 * Sg2;
  float SM2x = S11 * M21 + S12 * M22, SM2y = S12 * M21 + S22 * M22;
  float M2SM2 = M21 * SM2x + M22 * SM2y, M2Sg = M21 * Sg1 + M22 * Sg2;
  float Xc = -(r2 * M1Sg) / den;
  float hx = std::sqrt(Xc * Xc + (r2 * M1SM1) / den);
  float Yc = -(r2 * M2Sg) / den;
  float hy = std::sqrt(Yc * Yc + (r2 * M2SM2) / den);
  float xlo = ((x0 + Xc) - hx) - 0.01f, xhi = ((x0 + Xc) + hx) + 0.01f;
  float ylo = ((y0 + Yc) - hy) - 0.01f, yhi = ((y0 + Yc) + hy) + 0.01f;
  if (!(xlo <= xhi) || !(ylo <= yhi)) return b;
  float il = std::ceil(xlo - 0.5f), ih = std::floor(xhi - 0.5f);
  float jl = std::ceil(ylo - 0.5f), jh = std::floor(yhi - 0.5f);
  il = std::max(il, 0.f); ih = std::min(ih, (float)(cd.W - 1));
  jl = std::max(jl, 0.f); jh = std::min(jh, (float)(cd.H - 1));
  if (!(il <= ih) || !(jl <= jh)) return b;
  b.stage = 4;
  b.keep = 1;
  b.il = (int)il; b.ih = (int)ih; b.jl = (int)jl; b.jh = (int)jh;
  b.tx0 = (int)il / od.tile_w; b.tx1 = (int)ih / od.tile_w;
  b.ty0 = (int)jl / od.tile_h; b.ty1 = (int)jh / od.tile_h;
  return b;
}

// ------------------------------------------------------------ FP64 cull
// The cull rule (the bounding-rectangle reading of App. A.1): a surfel is kept
// when its whole MIP acceptance ellipse {u^T Sigma_mip^{-1} u < r_cut^2} lies
// beyond the near plane, i.e. its projection is a bounded ellipse.  The
// camera-space depth is linear along the surfel plane,
// z(u, v) = c'_z + u t'_uz + v t'_vz, so its minimum over the ellipse is
// c'_z - r_cut sqrt(t_z^T Sigma_mip t_z) with t_z = (t'_uz, t'_vz) (the support
// function of an ellipse).  Evaluated in FP64 from the oracle's own T rows and
// filter, independently of the FP32 binning decision.
// margin: (minimum depth - znear) / c'_z.
template <class S>
static bool cull_keep64(const Rec<S>& r, double znear, double rcut, double* margin) {
  const double z = val(r.T4[2]);
  if (!(z > znear)) {
    *margin = (z - znear) / std::max(std::fabs(z), 1e-300);
    return false;
  }
  const double a = val(r.T4[0]), b = val(r.T4[1]);
  const double q = a * a * val(r.sig[0]) + 2.0 * a * b * val(r.sig[1]) + b * b * val(r.sig[2]);
  const double zmin = z - rcut * std::sqrt(q);
  if (!std::isfinite(zmin)) {
    *margin = -INFINITY;
    return false;
  }
  *margin = (zmin - znear) / z;
  return zmin > znear;
}

// ------------------------------------------------------------ tone map
// The transfer applied to HDR images with eq:photo_loss (Sec. 3.7.1): log
// space, then the sRGB encoding (IEC 61966-2-1: linear segment 12.92 v up to
// v = 0.0031308, else 1.055 v^(1/2.4) - 0.055).  Negative inputs map to 0.
template <class S> static S tonemap_srgb_log(S x) {
  if (!(val(x) > 0.0)) return S(0.0);
  S v = log1p(x);
  if (val(v) <= 0.0031308) return 12.92 * v;
  return 1.055 * pow(v, 1.0 / 2.4) - 0.055;
}

// ------------------------------------------------------------ per pixel
// Ray-surfel intersection (Sec. 3.1), MIP-filtered weight (eq:mip_weight),
// interval grouping (Alg. 1), Shepard normalisation (eq:shepard), coverage
// opacity (eq:alpha), front-to-back compositing (eq:compositing), K_max cap
// (App. A.1), background blend and soft silhouette 1 - T_{K+1} (Sec. 3.5.2).
template <class S> struct Frag { double zs; int idx; S w; S ze; const Rec<S>* r; S z; };
// cons: the pixel's depth-consolidation term (eq:cons_loss), inter-layer plus
// intra-layer part, over the composited layers.
// depth: the composited layer depth sum_k T_k alpha_k z_k (alpha-weighted; the
// background contributes nothing).
// nf: fragments accumulated into the composited layers
template <class S> struct PixOut { S img[3]; S alpha; S cons; S depth; int nl; int nf = 0; };
// Fragments the per-pixel MIP filter accepts outside its support rectangle.
struct Dropped { int n = 0; double w = 0.0; };
// gap_margin: the closest depth-gap decision, and (t_min > 0) the closest
// early-out decision |T - t_min| / t_min.
struct PixDiag { double cut_margin = INFINITY, gap_margin = INFINITY; Dropped pp_drop; };

// zf (nullable): camera-space depth of the ray-surfel intersection,
// T4 . (u, v, 1) = c'_z + u t'_uz + v t'_vz.
template <class S>
static S frag_weight(const Rec<S>& r, double x, double y, double rc2, bool& hit, double& q_val,
                     S* zf = nullptr) {
  // clip-space planes h_x = (-1,0,0,x), h_y = (0,-1,0,y) mapped by T^T
  S k[3], l[3];
  for (int i = 0; i < 3; ++i) { k[i] = x * r.T4[i] - r.T1[i]; l[i] = y * r.T4[i] - r.T2[i]; }
  S p1 = k[1] * l[2] - k[2] * l[1];
  S p2 = k[2] * l[0] - k[0] * l[2];
  S p3 = k[0] * l[1] - k[1] * l[0];
  hit = false;
  q_val = INFINITY;
  if (val(p3) == 0.0) return S(0.0);
  S u = p1 / p3, v = p2 / p3;
  S h = r.T4[0] * u + r.T4[1] * v + r.T4[2];
  if (val(h) <= 0.0) return S(0.0);  // behind the eye
  if (zf) *zf = h;
  S q = r.sinv[0] * u * u + 2.0 * r.sinv[1] * u * v + r.sinv[2] * v * v;
  q_val = val(q);
  if (!(q_val < rc2)) return S(0.0);
  hit = true;
  using std::exp;
  return r.nf * exp(-0.5 * q);
}

// Per-pixel MIP variant (Sec. 3.3.1, the formulation the centre precomputation
// approximates): the Jacobian J = d(u,v)/d(x,y) of the ray-surfel
// intersection is taken at this pixel's intersection (quotient rule on
// u = p1/p3, v = p2/p3 with dp/dx = T4 x l, dp/dy = k x T4), then
// Sigma_mip = I + sigma_f J J^T, q = u^T Sigma_mip^{-1} u, n_f = |Sigma_mip|^{-1/2}.
// Reading: the support stays the FP32 binning rectangle of the centre filter
// (the variant runs inside the same binning) intersected with q < r_cut^2.
// dropped (nullable): counts (and sums the weights of) the fragments the
// per-pixel filter accepts (q < r_cut^2) at pixels outside that rectangle, i.e.
// the fragments this support reading removes.
template <class S>
static S frag_weight_pp(const Rec<S>& r, double x, double y, double rc2, double sigma_f, bool& hit,
                        double& q_val, S* zf = nullptr, Dropped* dropped = nullptr) {
  using std::sqrt;
  using std::exp;
  hit = false;
  q_val = INFINITY;
  const int px = (int)std::floor(x), py = (int)std::floor(y);
  const bool in_rect = !(px < r.rect[0] || px > r.rect[1] || py < r.rect[2] || py > r.rect[3]);
  if (!in_rect && !dropped) return S(0.0);
  S k[3], l[3];
  for (int i = 0; i < 3; ++i) { k[i] = x * r.T4[i] - r.T1[i]; l[i] = y * r.T4[i] - r.T2[i]; }
  S p1 = k[1] * l[2] - k[2] * l[1];
  S p2 = k[2] * l[0] - k[0] * l[2];
  S p3 = k[0] * l[1] - k[1] * l[0];
  if (val(p3) == 0.0) return S(0.0);
  S u = p1 / p3, v = p2 / p3;
  S h = r.T4[0] * u + r.T4[1] * v + r.T4[2];
  if (val(h) <= 0.0) return S(0.0);
  if (zf) *zf = h;
  // dp/dx = T4 x l, dp/dy = k x T4
  S px1 = r.T4[1] * l[2] - r.T4[2] * l[1], px2 = r.T4[2] * l[0] - r.T4[0] * l[2],
    px3 = r.T4[0] * l[1] - r.T4[1] * l[0];
  S py1 = k[1] * r.T4[2] - k[2] * r.T4[1], py2 = k[2] * r.T4[0] - k[0] * r.T4[2],
    py3 = k[0] * r.T4[1] - k[1] * r.T4[0];
  S Jux = (px1 - u * px3) / p3, Juy = (py1 - u * py3) / p3;
  S Jvx = (px2 - v * px3) / p3, Jvy = (py2 - v * py3) / p3;
  S s11 = 1.0 + sigma_f * (Jux * Jux + Juy * Juy);
  S s12 = sigma_f * (Jux * Jvx + Juy * Jvy);
  S s22 = 1.0 + sigma_f * (Jvx * Jvx + Jvy * Jvy);
  S det = s11 * s22 - s12 * s12;
  S q = (s22 * u * u - 2.0 * s12 * u * v + s11 * v * v) / det;
  if (!in_rect) {
    if (val(q) < rc2) {
      ++dropped->n;
      dropped->w += std::sqrt(1.0 / val(det)) * std::exp(-0.5 * val(q));
    }
    return S(0.0);
  }
  q_val = val(q);
  if (!(q_val < rc2)) return S(0.0);
  hit = true;
  return sqrt(1.0 / det) * exp(-0.5 * q);
}

template <class S>
static void pixel_eval(double x, double y, const Rec<S>* recs, const std::vector<int>& cand,
                       const Cam& cam, const Opt& o, PixOut<S>& out, PixDiag* dg,
                       std::vector<int>* covering, std::vector<int>* layer_of = nullptr,
                       std::vector<double>* wout = nullptr) {
  using std::exp;
  using std::sqrt;
  const double rc2 = o.r_cut * o.r_cut;
  std::vector<Frag<S>> fr;
  double cm = INFINITY;
  for (int i : cand) {
    bool hit;
    double q;
    S z(0.0);
    S w = o.mip == 1 ? frag_weight_pp(recs[i], x, y, rc2, o.sigma_f, hit, q, &z, dg ? &dg->pp_drop : nullptr)
                     : frag_weight(recs[i], x, y, rc2, hit, q, &z);
    if (std::isfinite(q)) cm = std::min(cm, std::fabs(q - rc2) / rc2);
    if (!hit) continue;
    fr.push_back({val(recs[i].zs), i, w, recs[i].ze, &recs[i], z});
  }
  std::sort(fr.begin(), fr.end(), [](const Frag<S>& a, const Frag<S>& b) {
    return a.zs < b.zs || (a.zs == b.zs && a.idx < b.idx);
  });
  if (covering) { covering->clear(); for (auto& f : fr) covering->push_back(f.idx); }
  if (layer_of) layer_of->assign(fr.size(), -1);
  if (wout) { wout->clear(); for (auto& f : fr) wout->push_back(val(f.w)); }
  const double kappa = o.gamma / (2.0 * kPi);
  S Cg[3] = {S(0.0), S(0.0), S(0.0)}, Wg = S(0.0);
  double zmax = 0.0;
  S Cout[3] = {S(0.0), S(0.0), S(0.0)}, Tb = S(1.0);
  int K = 0;
  double gm = INFINITY;
  // depth statistics of the layers (eq:cons_loss): compositing weight
  // T_k alpha_k, Shepard-weighted mean depth and variance of the fragments
  std::vector<const Frag<S>*> members;
  std::vector<S> lw, lz, lv;
  auto flush = [&]() {
    S a = 1.0 - exp(-kappa * Wg);
    if (o.shade == 2) {
      // normal image (Sec. 4.2.3): the Shepard mean of the unit normals,
      // renormalised to unit length, per layer
      S nrm = sqrt(Cg[0] * Cg[0] + Cg[1] * Cg[1] + Cg[2] * Cg[2]);
      for (int c = 0; c < 3; ++c) Cout[c] += Tb * a * (Cg[c] / nrm);
    } else {
      for (int c = 0; c < 3; ++c) Cout[c] += Tb * a * (Cg[c] / Wg);
    }
    S zm(0.0), var(0.0);
    for (const Frag<S>* f : members) zm += f->w * f->z;
    zm = zm / Wg;
    for (const Frag<S>* f : members) var += f->w * (f->z - zm) * (f->z - zm);
    var = var / Wg;
    lw.push_back(Tb * a);
    lz.push_back(zm);
    lv.push_back(var);
    members.clear();
    Tb = Tb * (1.0 - a);
    ++K;
  };
  bool done = false;
  for (size_t fi = 0; fi < fr.size(); ++fi) {
    auto& f = fr[fi];
    if (val(Wg) > 0.0) {
      gm = std::min(gm, std::fabs(f.zs - zmax) / std::max(std::fabs(zmax), 1e-300));
      if (f.zs > zmax) {  // gap detected: finalise the current layer
        flush();
        if (o.t_min > 0.0) gm = std::min(gm, std::fabs(val(Tb) - o.t_min) / o.t_min);
        // the K_max cap (App. A.1), or the early-out once the transmittance in
        // front of the next layer is below t_min
        if (K >= o.k_max || val(Tb) < o.t_min) { done = true; break; }
        Cg[0] = Cg[1] = Cg[2] = S(0.0);
        Wg = S(0.0);
        zmax = 0.0;
      }
    }
    zmax = std::max(zmax, val(f.ze));
    ++out.nf;
    if (layer_of) (*layer_of)[fi] = K;
    for (int c = 0; c < 3; ++c) Cg[c] += f.w * f.r->col[c];
    Wg += f.w;
    members.push_back(&f);
  }
  if (!done && val(Wg) > 0.0) flush();
  for (int c = 0; c < 3; ++c) {
    out.img[c] = Cout[c] + Tb * cam.bg[c];
    if (o.tonemap) out.img[c] = tonemap_srgb_log(out.img[c]);
  }
  out.alpha = 1.0 - Tb;
  S cons(0.0);
  for (int i = 0; i < K; ++i) {
    for (int j = i + 1; j < K; ++j) {
      S d = lz[i] - lz[j];
      cons += lw[i] * lw[j] * (val(d) >= 0.0 ? d : -d);
    }
    cons += lw[i] * lw[i] * lv[i];
  }
  out.cons = cons;
  S depth(0.0);
  for (int i = 0; i < K; ++i) depth += lw[i] * lz[i];
  out.depth = depth;
  out.nl = K;
  if (dg) { dg->cut_margin = cm; dg->gap_margin = gm; }
}

// ------------------------------------------------------------ scene loading
template <class S>
static Surf<S> load_surf(const float* const* P, int n, int i, const double* const* V) {
  Surf<S> s;
  auto get = [&](int a, int k) -> S {
    double x = P[a][(size_t)k * n + i];
    if constexpr (std::is_same<S, Dual>::value) {
      return Dual(x, V && V[a] ? V[a][(size_t)k * n + i] : 0.0);
    } else {
      return S(x);
    }
  };
  for (int k = 0; k < 3; ++k) { s.p[k] = get(0, k); s.n[k] = get(1, k); s.t[k] = get(2, k); s.alb[k] = get(4, k); }
  s.s[0] = get(3, 0); s.s[1] = get(3, 1);
  s.rough = get(5, 0);
  s.metal = get(6, 0);
  return s;
}

// Per-surfel quantities of one view: FP64 records of every surfel, the FP32
// binning decision (kept for the comparison with the GPU binning and for the
// support of the per-pixel MIP variant), the FP64 cull (keep) and the candidate
// list = the surfels the FP64 cull keeps.  The FP32 decision does not choose
// the candidates: a covering fragment of a surfel that it culls, or outside its
// FP32 pixel rectangle, is a bounding-rectangle violation.
template <class S, class M>
static void prepare(const float* const* P, int n, const double* const* V, const Cam& c, const Opt& o,
                    const M& maps, const MapDims* md, const Lut* L, std::vector<Rec<S>>& recs,
                    std::vector<BinOut>& bins, std::vector<int>& keep, std::vector<int>& cand,
                    std::vector<double>* margin = nullptr) {
  recs.assign(n, Rec<S>());
  bins.assign(n, BinOut{0, 0, 0.f, 0, 0, -1, -1, 0, -1, 0, -1});
  keep.assign(n, 0);
  if (margin) margin->assign(n, 0.0);
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i) {
    bins[i] = bin_f32(P, n, i, c, o);
    Surf<S> s = load_surf<S>(P, n, i, V);
    preprocess(s, c, o, maps, md, L, recs[i]);
    set_rect(recs[i], bins[i]);
    double m = 0.0;
    keep[i] = cull_keep64(recs[i], c.znear, o.r_cut, &m) ? 1 : 0;
    if (margin) (*margin)[i] = m;
  }
  cand.clear();
  for (int i = 0; i < n; ++i)
    if (keep[i]) cand.push_back(i);
}

// Is pixel (px, py) outside the FP32 binning of surfel i (culled, or outside
// its inclusive pixel rectangle)?
static bool outside_bin(const BinOut& b, int px, int py) {
  return !b.keep || px < b.il || px > b.ih || py < b.jl || py > b.jh;
}

}  // namespace orc

using namespace orc;

extern "C" {

// Environment-map prefilter (eq:ibl, Sec. 3.4.2; conventions are this
// implementation's reading of the silent points).  maps: flat layout of MapDims.
int orc_envmap_size(int He, int We) { return (int)MapDims(He, We).total(); }
int orc_envmap(const double* E, int He, int We, double* maps) {
  envmap_prefilter<double>(E, He, We, maps);
  return 0;
}
int orc_envmap_adjoint(const double* dmaps, int He, int We, double* dE) {
  envmap_adjoint(dmaps, He, We, dE);
  return 0;
}
// Threads of the OpenMP loops (n > 0 sets it); returns the count in use.
int orc_set_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
}

int orc_brdf_lut(int n_nv, int n_r, int samples, double* out) {
  brdf_lut(n_nv, n_r, samples, out);
  return 0;
}

// FP32 binning reference.  P: the 7 parameter arrays (position, normal, tangent,
// scale, albedo, roughness, metallic; [C][n] float32).  Outputs per surfel:
// keep, z_start (float bits), inclusive tile rectangle (tx0, ty0, tx1, ty1) and
// (pixel_rect, nullable) the inclusive pixel rectangle (il, ih, jl, jh).
int orc_bin_f32(const float* const* P, int n, const double* cam, const double* opt,
                int* keep, uint32_t* zbits, int* rect, int* pixel_rect) {
  Cam c = unpack_cam(cam);
  Opt o = unpack_opt(opt);
  for (int i = 0; i < n; ++i) {
    BinOut b = bin_f32(P, n, i, c, o);
    keep[i] = b.keep;
    std::memcpy(&zbits[i], &b.zs, 4);
    rect[4 * i + 0] = b.tx0; rect[4 * i + 1] = b.ty0;
    rect[4 * i + 2] = b.tx1; rect[4 * i + 3] = b.ty1;
    if (pixel_rect) {
      pixel_rect[4 * i + 0] = b.il; pixel_rect[4 * i + 1] = b.ih;
      pixel_rect[4 * i + 2] = b.jl; pixel_rect[4 * i + 3] = b.jh;
    }
  }
  return 0;
}

// Forward.  maps: flat map set (NULL in albedo mode); lut [n_r][n_nv][2].
// pix: npix (x, y) integer pixel indices; pixel centres at (x + 1/2, y + 1/2).
// Outputs per listed pixel: image [3], alpha, layer count, decision margins
// (cutoff |q - r^2|/r^2 and gap |z_start - z_max|/z_max, minimum over the
// pixel), the number of covering fragments outside the FP32 tile rectangle and
// (cons, nullable) the depth-consolidation term of eq:cons_loss and (depth,
// nullable) the composited depth sum_k T_k alpha_k z_k.
int orc_render(const float* const* P, int n, const double* cam, const double* opt,
               const double* maps, int He, int We, const double* lut, int n_nv, int n_r,
               int npix, const int* pix, double* img, double* alpha, int* nl,
               double* cut_margin, double* gap_margin, int* viol, double* cons, double* depth,
               int* pp_drop, double* pp_drop_w, int* nfrag) {
  Cam c = unpack_cam(cam);
  Opt o = unpack_opt(opt);
  std::vector<Rec<double>> recs;
  std::vector<BinOut> bins;
  std::vector<int> keep, cand;
  MapDims md(std::max(He, 4), std::max(We, 8));
  Lut L{lut, n_nv, n_r};
  MapsD M{maps};
  prepare(P, n, nullptr, c, o, M, &md, &L, recs, bins, keep, cand);
#pragma omp parallel for schedule(dynamic, 4)
  for (int k = 0; k < npix; ++k) {
    int px = pix[2 * k], py = pix[2 * k + 1];
    PixOut<double> out;
    PixDiag dg;
    std::vector<int> cov;
    pixel_eval(px + 0.5, py + 0.5, recs.data(), cand, c, o, out, &dg, &cov);
    int v = 0;
    for (int i : cov)
      if (outside_bin(bins[i], px, py)) ++v;
    for (int ch = 0; ch < 3; ++ch) img[3 * k + ch] = out.img[ch];
    alpha[k] = out.alpha;
    nl[k] = out.nl;
    cut_margin[k] = dg.cut_margin;
    gap_margin[k] = dg.gap_margin;
    viol[k] = v;
    if (cons) cons[k] = out.cons;
    if (depth) depth[k] = out.depth;
    if (pp_drop) pp_drop[k] = dg.pp_drop.n;
    if (nfrag) nfrag[k] = out.nf;
    if (pp_drop_w) pp_drop_w[k] = dg.pp_drop.w;
  }
  return 0;
}

// Directional derivative (exact, dual numbers) of the listed pixels' image,
// alpha, (cons_dot, nullable) depth-consolidation term and (depth_dot, nullable)
// composited depth along the parameter
// direction V (7 arrays, NULL = 0) and the map-set direction dmaps (NULL = 0).
int orc_render_jvp(const float* const* P, int n, const double* const* V, const double* cam,
                   const double* opt, const double* maps, const double* dmaps, int He, int We,
                   const double* lut, int n_nv, int n_r, int npix, const int* pix,
                   double* img, double* img_dot, double* alpha_dot, double* cons_dot,
                   double* depth_dot) {
  Cam c = unpack_cam(cam);
  Opt o = unpack_opt(opt);
  std::vector<Rec<Dual>> recs;
  std::vector<BinOut> bins;
  std::vector<int> keep, cand;
  MapDims md(std::max(He, 4), std::max(We, 8));
  Lut L{lut, n_nv, n_r};
  MapsDual M{maps, dmaps};
  prepare(P, n, V, c, o, M, &md, &L, recs, bins, keep, cand);
#pragma omp parallel for schedule(dynamic, 4)
  for (int k = 0; k < npix; ++k) {
    PixOut<Dual> out;
    pixel_eval(pix[2 * k] + 0.5, pix[2 * k + 1] + 0.5, recs.data(), cand, c, o, out, nullptr, nullptr);
    for (int ch = 0; ch < 3; ++ch) { img[3 * k + ch] = out.img[ch].v; img_dot[3 * k + ch] = out.img[ch].d; }
    alpha_dot[k] = out.alpha.d;
    if (cons_dot) cons_dot[k] = out.cons.d;
    if (depth_dot) depth_dot[k] = out.depth.d;
  }
  return 0;
}

// Adjoint.  Given dL/dimage [npix][3], dL/dalpha [npix] (nullable), dL/dcons
// [npix] (nullable; cons = eq:cons_loss per pixel) and dL/ddepth [npix]
// (nullable) at the listed pixels, accumulate dL/dparams (7 arrays, [C][n] double, overwritten)
// and dL/dmaps (flat map set, overwritten; the environment itself is then
// reached through orc_envmap_adjoint).  Reverse mode on a tape, per pixel for
// the rasterisation and per surfel for preprocessing and shading.
int orc_render_grad(const float* const* P, int n, const double* cam, const double* opt,
                    const double* maps, int He, int We, const double* lut, int n_nv, int n_r,
                    int npix, const int* pix, const double* dimg, const double* dalpha,
                    double* const* dP, double* dmaps, const double* dcons, const double* ddepth) {
  Cam c = unpack_cam(cam);
  Opt o = unpack_opt(opt);
  std::vector<Rec<double>> recs;
  std::vector<BinOut> bins;
  std::vector<int> keep, cand;
  MapDims md(std::max(He, 4), std::max(We, 8));
  Lut L{lut, n_nv, n_r};
  MapsD Md{maps};
  const int csz[7] = {3, 3, 3, 2, 3, 1, 1};
  for (int a = 0; a < 7; ++a)
    if (dP[a]) std::fill(dP[a], dP[a] + (size_t)csz[a] * n, 0.0);
  if (dmaps && He > 0) std::fill(dmaps, dmaps + md.total(), 0.0);
  prepare(P, n, nullptr, c, o, Md, &md, &L, recs, bins, keep, cand);
  // adjoint of each record: T1, T2, T4 (9), zs, ze (no gradient), sinv (3), nf, col (3)
  const int NR = 16;
  std::vector<double> drec((size_t)n * NR, 0.0);
#pragma omp parallel
  {
    Tape tape;
    g_tape = &tape;
    std::vector<int> cov;
#pragma omp for schedule(dynamic, 4)
    for (int k = 0; k < npix; ++k) {
      double x = pix[2 * k] + 0.5, y = pix[2 * k + 1] + 0.5;
      PixOut<double> od;
      pixel_eval(x, y, recs.data(), cand, c, o, od, nullptr, &cov);
      if (cov.empty()) continue;
      tape.clear();
      // leaves for the covering records only; the other records do not reach
      // the pixel (identical decisions: the values are the same doubles)
      std::vector<Rec<Var>> vr(cov.size());
      std::unordered_map<int, int> slot;
      for (size_t j = 0; j < cov.size(); ++j) {
        const Rec<double>& r = recs[cov[j]];
        Rec<Var>& v = vr[j];
        for (int a = 0; a < 3; ++a) { v.T1[a] = Var::leaf(r.T1[a]); v.T2[a] = Var::leaf(r.T2[a]); v.T4[a] = Var::leaf(r.T4[a]); }
        v.zs = Var(r.zs); v.ze = Var(r.ze);
        for (int a = 0; a < 4; ++a) v.rect[a] = r.rect[a];
        for (int a = 0; a < 3; ++a) v.sinv[a] = Var::leaf(r.sinv[a]);
        v.nf = Var::leaf(r.nf);
        for (int a = 0; a < 3; ++a) v.col[a] = Var::leaf(r.col[a]);
        slot[cov[j]] = (int)j;
      }
      // evaluate with Var records laid out densely; candidate list = slots
      std::vector<int> dense(cov.size());
      for (size_t j = 0; j < cov.size(); ++j) dense[j] = (int)j;
      PixOut<Var> ov;
      pixel_eval(x, y, vr.data(), dense, c, o, ov, nullptr, nullptr);
      std::vector<double> adj(tape.nodes.size(), 0.0);
      for (int ch = 0; ch < 3; ++ch)
        if (ov.img[ch].id >= 0) adj[ov.img[ch].id] += dimg[3 * k + ch];
      if (dalpha && ov.alpha.id >= 0) adj[ov.alpha.id] += dalpha[k];
      if (dcons && ov.cons.id >= 0) adj[ov.cons.id] += dcons[k];
      if (ddepth && ov.depth.id >= 0) adj[ov.depth.id] += ddepth[k];
      tape.sweep(adj);
      for (size_t j = 0; j < cov.size(); ++j) {
        const Rec<Var>& v = vr[j];
        const Var* f[NR] = {&v.T1[0], &v.T1[1], &v.T1[2], &v.T2[0], &v.T2[1], &v.T2[2],
                            &v.T4[0], &v.T4[1], &v.T4[2], &v.sinv[0], &v.sinv[1], &v.sinv[2],
                            &v.nf, &v.col[0], &v.col[1], &v.col[2]};
        double* dst = &drec[(size_t)cov[j] * NR];
        for (int a = 0; a < NR; ++a) {
          double g = adj[f[a]->id];
          if (g != 0.0) {
#pragma omp atomic
            dst[a] += g;
          }
        }
      }
    }
    g_tape = nullptr;
  }
  // per surfel: reverse through preprocessing and shading
#pragma omp parallel
  {
    Tape tape;
    g_tape = &tape;
#pragma omp for schedule(dynamic, 64)
    for (int i = 0; i < n; ++i) {
      if (!keep[i]) continue;
      const double* dr = &drec[(size_t)i * NR];
      bool any = false;
      for (int a = 0; a < NR; ++a) any |= dr[a] != 0.0;
      if (!any) continue;
      tape.clear();
      Surf<Var> s;
      for (int k = 0; k < 3; ++k) {
        s.p[k] = Var::leaf(P[0][(size_t)k * n + i]);
        s.n[k] = Var::leaf(P[1][(size_t)k * n + i]);
        s.t[k] = Var::leaf(P[2][(size_t)k * n + i]);
        s.alb[k] = Var::leaf(P[4][(size_t)k * n + i]);
      }
      s.s[0] = Var::leaf(P[3][i]); s.s[1] = Var::leaf(P[3][(size_t)n + i]);
      s.rough = Var::leaf(P[5][i]);
      s.metal = Var::leaf(P[6][i]);
      MapsVar Mv{maps, {}};
      Rec<Var> r;
      preprocess(s, c, o, Mv, &md, &L, r);
      std::vector<double> adj(tape.nodes.size(), 0.0);
      const Var* f[NR] = {&r.T1[0], &r.T1[1], &r.T1[2], &r.T2[0], &r.T2[1], &r.T2[2],
                          &r.T4[0], &r.T4[1], &r.T4[2], &r.sinv[0], &r.sinv[1], &r.sinv[2],
                          &r.nf, &r.col[0], &r.col[1], &r.col[2]};
      for (int a = 0; a < NR; ++a)
        if (f[a]->id >= 0) adj[f[a]->id] += dr[a];
      tape.sweep(adj);
      auto put = [&](int arr, int k, const Var& v) {
        if (dP[arr] && v.id >= 0) dP[arr][(size_t)k * n + i] += adj[v.id];
      };
      for (int k = 0; k < 3; ++k) { put(0, k, s.p[k]); put(1, k, s.n[k]); put(2, k, s.t[k]); put(4, k, s.alb[k]); }
      put(3, 0, s.s[0]); put(3, 1, s.s[1]);
      put(5, 0, s.rough); put(6, 0, s.metal);
      if (dmaps && He > 0)
        for (auto& kv : Mv.used) {
          double g = adj[kv.second.id];
          if (g != 0.0) {
#pragma omp atomic
            dmaps[kv.first] += g;
          }
        }
    }
    g_tape = nullptr;
  }
  return 0;
}

// Densification statistic (Sec. 3.6.1, eq:ss_grad).  For each listed pixel p
// with loss L_p = dimg_p . image_p + dalpha_p alpha_p (+ dcons_p cons_p, the
// depth-consolidation term, when dcons is given) and each surfel i that
// reaches p, the screen-space positional gradient is
//   g = (dL_p/dT1z * T4z, dL_p/dT2z * T4z),
// with the whole pixel evaluation, MIP filter included, differentiated as a
// function of the T rows.  Outputs per surfel (overwritten): the sum over the
// pixels of |g| (abs_sum [n]), of g itself (vec_sum [2][n], nullable) and
// whether the surfel survives the cull with a non-empty tile rectangle in this
// view (visible [n], nullable).  The paper's criterion averages abs_sum over
// the views in which a surfel is visible.
int orc_screen_grad(const float* const* P, int n, const double* cam, const double* opt,
                    const double* maps, int He, int We, const double* lut, int n_nv, int n_r,
                    int npix, const int* pix, const double* dimg, const double* dalpha,
                    double* abs_sum, double* vec_sum, int* visible, const double* dcons) {
  Cam c = unpack_cam(cam);
  Opt o = unpack_opt(opt);
  std::vector<Rec<double>> recs;
  std::vector<BinOut> bins;
  std::vector<int> keep, cand;
  MapDims md(std::max(He, 4), std::max(We, 8));
  Lut L{lut, n_nv, n_r};
  MapsD Md{maps};
  prepare(P, n, nullptr, c, o, Md, &md, &L, recs, bins, keep, cand);
  for (int i = 0; i < n; ++i) {
    abs_sum[i] = 0.0;
    if (vec_sum) vec_sum[i] = vec_sum[(size_t)n + i] = 0.0;
    // the views a surfel "contributed" to: the binning decision (cull and a
    // non-empty rectangle)
    if (visible) visible[i] = bins[i].keep;
  }
#pragma omp parallel
  {
    Tape tape;
    g_tape = &tape;
    std::vector<int> cov;
#pragma omp for schedule(dynamic, 4)
    for (int k = 0; k < npix; ++k) {
      double x = pix[2 * k] + 0.5, y = pix[2 * k + 1] + 0.5;
      PixOut<double> od;
      pixel_eval(x, y, recs.data(), cand, c, o, od, nullptr, &cov);
      if (cov.empty()) continue;
      tape.clear();
      // leaves: the T rows and the colour; the MIP filter is rebuilt from T
      std::vector<Rec<Var>> vr(cov.size());
      for (size_t j = 0; j < cov.size(); ++j) {
        const Rec<double>& r = recs[cov[j]];
        Rec<Var>& v = vr[j];
        for (int a = 0; a < 3; ++a) { v.T1[a] = Var::leaf(r.T1[a]); v.T2[a] = Var::leaf(r.T2[a]); v.T4[a] = Var::leaf(r.T4[a]); }
        v.zs = Var(r.zs); v.ze = Var(r.ze);
        for (int a = 0; a < 4; ++a) v.rect[a] = r.rect[a];
        mip_filter(v, o.sigma_f);
        for (int a = 0; a < 3; ++a) v.col[a] = Var::leaf(r.col[a]);
      }
      std::vector<int> dense(cov.size());
      for (size_t j = 0; j < cov.size(); ++j) dense[j] = (int)j;
      PixOut<Var> ov;
      pixel_eval(x, y, vr.data(), dense, c, o, ov, nullptr, nullptr);
      std::vector<double> adj(tape.nodes.size(), 0.0);
      for (int ch = 0; ch < 3; ++ch)
        if (ov.img[ch].id >= 0) adj[ov.img[ch].id] += dimg[3 * k + ch];
      if (dalpha && ov.alpha.id >= 0) adj[ov.alpha.id] += dalpha[k];
      if (dcons && ov.cons.id >= 0) adj[ov.cons.id] += dcons[k];
      tape.sweep(adj);
      for (size_t j = 0; j < cov.size(); ++j) {
        const int i = cov[j];
        const double t4z = recs[i].T4[2];
        const double gx = adj[vr[j].T1[2].id] * t4z, gy = adj[vr[j].T2[2].id] * t4z;
        const double a = std::sqrt(gx * gx + gy * gy);
#pragma omp atomic
        abs_sum[i] += a;
        if (vec_sum) {
#pragma omp atomic
          vec_sum[i] += gx;
#pragma omp atomic
          vec_sum[(size_t)n + i] += gy;
        }
      }
    }
    g_tape = nullptr;
  }
  return 0;
}

// Debug view of one pixel: the covering fragments in the order the grouping
// visits them, with record index, z_start, z_end, weight and layer (-1 when
// discarded after the K_max-th layer).  Returns the fragment count (at most cap
// entries are written).
int orc_pixel_fragments(const float* const* P, int n, const double* cam, const double* opt,
                        const double* maps, int He, int We, const double* lut, int n_nv, int n_r,
                        int px, int py, int cap, int* idx, double* zs, double* ze, double* w,
                        int* layer) {
  Cam c = unpack_cam(cam);
  Opt o = unpack_opt(opt);
  std::vector<Rec<double>> recs;
  std::vector<BinOut> bins;
  std::vector<int> keep, cand;
  MapDims md(std::max(He, 4), std::max(We, 8));
  Lut L{lut, n_nv, n_r};
  MapsD M{maps};
  prepare(P, n, nullptr, c, o, M, &md, &L, recs, bins, keep, cand);
  PixOut<double> out;
  std::vector<int> cov, lay;
  std::vector<double> ws;
  pixel_eval(px + 0.5, py + 0.5, recs.data(), cand, c, o, out, nullptr, &cov, &lay, &ws);
  for (size_t j = 0; j < cov.size() && (int)j < cap; ++j) {
    idx[j] = cov[j];
    zs[j] = recs[cov[j]].zs;
    ze[j] = recs[cov[j]].ze;
    w[j] = ws[j];
    layer[j] = lay[j];
  }
  return (int)cov.size();
}

// Per-surfel records of one view (test access): 26 doubles per surfel:
// T1 (3), T2 (3), T4 (3), z_start, z_end, Sigma_mip^{-1} (3), Sigma_mip (3), n_f,
// FP64 keep, FP64 cull margin (see cull_keep64), FP32 keep, FP32 pixel
// rectangle il, ih, jl, jh, FP32 binning stage (see BinOut).
int orc_records(const float* const* P, int n, const double* cam, const double* opt, double* out) {
  Cam c = unpack_cam(cam);
  Opt o = unpack_opt(opt);
  std::vector<Rec<double>> recs;
  std::vector<BinOut> bins;
  std::vector<int> keep, cand;
  std::vector<double> margin;
  MapDims md(4, 8);
  std::vector<double> zero_maps(md.total(), 0.0), zero_lut(8, 0.0);
  Lut L{zero_lut.data(), 2, 2};
  MapsD M{zero_maps.data()};
  Opt oa = o;
  oa.shade = 0;  // geometry only
  prepare(P, n, nullptr, c, oa, M, &md, &L, recs, bins, keep, cand, &margin);
  for (int i = 0; i < n; ++i) {
    double* d = out + (size_t)i * 26;
    const Rec<double>& r = recs[i];
    for (int a = 0; a < 3; ++a) { d[a] = r.T1[a]; d[3 + a] = r.T2[a]; d[6 + a] = r.T4[a]; }
    d[9] = r.zs; d[10] = r.ze;
    for (int a = 0; a < 3; ++a) { d[11 + a] = r.sinv[a]; d[14 + a] = r.sig[a]; }
    d[17] = r.nf;
    d[18] = keep[i];
    d[19] = margin[i];
    d[20] = bins[i].keep;
    d[21] = bins[i].il; d[22] = bins[i].ih; d[23] = bins[i].jl; d[24] = bins[i].jh;
    d[25] = bins[i].stage;
  }
  return 0;
}

}  // extern "C"
