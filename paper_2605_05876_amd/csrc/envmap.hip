// Environment-map levels for split-sum shading (eq:ibl, Sec. 3.4.2) and their
// adjoint, plus the BRDF scale/bias table.
//
// Levels of a scene: 0 = E (H_e x W_e), 1..5 = GGX-prefiltered with
// alpha_l = (l/5)^2 at max(H_e >> l, 4) x max(W_e >> l, 8), 6 = irradiance
// (32 x 64).  With input texel directions d_t and exact solid angles dO_t:
//   Irr(d)   = (1/pi) sum_t E_t max(0, d.d_t) dO_t
//   Spec_l(R) = sum_t E_t K_l(R,t) / sum_t K_l(R,t),
//   K_l(R,t) = D(R.h_t; alpha_l) max(0, R.d_t) dO_t,  h_t = (R + d_t)/|R + d_t|,
// the split-sum prefilter with n = v = R.  For unit R and d_t,
// (R.h_t)^2 = (1 + R.d_t)/2, so D needs only the cosine.
#include "common.h"

namespace ss {

__device__ inline void texel_dir(int a, int b, int H, int W, float d[3]) {
  float th = kPi * ((float)a + 0.5f) / (float)H;
  float ph = 2.f * kPi * ((float)b + 0.5f) / (float)W;
  float st, ct, sp, cp;
  sincosf(th, &st, &ct);
  sincosf(ph, &sp, &cp);
  d[0] = st * cp;
  d[1] = st * sp;
  d[2] = ct;
}

// dirs[t] = (d_t, dOmega_t) for an H x W map
__global__ void envmap_dirs_kernel(float4* dirs, int H, int W) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= H * W) return;
  int a = i / W, b = i % W;
  float d[3];
  texel_dir(a, b, H, W, d);
  float dom = (2.f * kPi / (float)W) *
              (cosf(kPi * (float)a / (float)H) - cosf(kPi * (float)(a + 1) / (float)H));
  dirs[i] = make_float4(d[0], d[1], d[2], dom);
}

hipError_t launch_envmap_dirs(float* dirs, int H, int W, hipStream_t st) {
  int n = H * W;
  hipLaunchKernelGGL(envmap_dirs_kernel, dim3((n + 255) / 256), dim3(256), 0, st,
                     reinterpret_cast<float4*>(dirs), H, W);
  return hipGetLastError();
}

__device__ inline float ggx_weight(float c, float alpha) {
  // D(mu; alpha) max(0, c) with mu^2 = (1 + c)/2
  float a2 = alpha * alpha;
  float mu2 = 0.5f * (1.f + c);
  float t = mu2 * (a2 - 1.f) + 1.f;
  return a2 / (kPi * t * t) * c;
}

struct LevelSet {
  float* out[7];
  int h[7], w[7];
  int first[8];  // first output texel of each level in the flattened grid (levels 1..6)
};

__device__ inline int level_of(const int first[8], int o) {
  int l = 1;
  while (l < 6 && o >= first[l + 1]) ++l;
  return l;
}

// Output-texel table of levels 1..6 (built once per environment resolution):
// out_dirs[o] = (R, 1/Z) with Z = sum_t K_l(R,t) for the specular levels and
// Z = pi for the irradiance level.  Z does not depend on E.
__global__ void __launch_bounds__(256) envmap_out_dirs_kernel(int nt, const float4* __restrict__ dirs,
                                                              LevelSet L, float4* __restrict__ out_dirs) {
  __shared__ float red[256];
  const int o = blockIdx.x;
  const int l = level_of(L.first, o);
  const int k = o - L.first[l];
  const int W = L.w[l];
  float R[3];
  texel_dir(k / W, k % W, L.h[l], W, R);
  float z = 0.f;
  if (l < 6) {
    const float alpha = (float)(l * l) / 25.f;
    for (int t = threadIdx.x; t < nt; t += blockDim.x) {
      const float4 d = dirs[t];
      const float c = R[0] * d.x + R[1] * d.y + R[2] * d.z;
      if (c > 0.f) z += ggx_weight(c, alpha) * d.w;
    }
  }
  red[threadIdx.x] = z;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out_dirs[o] = make_float4(R[0], R[1], R[2], l < 6 ? 1.f / red[0] : 1.f / kPi);
}

// One block per output texel of levels 1..6; threads stride over the input
// texels, then a block reduction.
__global__ void __launch_bounds__(256) envmap_prefilter_kernel(const float* __restrict__ E, int nt,
                                                               const float4* __restrict__ dirs,
                                                               const float4* __restrict__ out_dirs,
                                                               LevelSet L) {
  __shared__ float red[3][256];
  const int o = blockIdx.x;
  const int l = level_of(L.first, o);
  const int k = o - L.first[l];
  const float4 R = out_dirs[o];
  float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f;
  if (l == 6) {
    for (int t = threadIdx.x; t < nt; t += blockDim.x) {
      const float4 d = dirs[t];
      const float c = R.x * d.x + R.y * d.y + R.z * d.z;
      if (c <= 0.f) continue;
      const float kk = c * d.w;
      acc0 += E[3 * t] * kk;
      acc1 += E[3 * t + 1] * kk;
      acc2 += E[3 * t + 2] * kk;
    }
  } else {
    const float alpha = (float)(l * l) / 25.f;
    for (int t = threadIdx.x; t < nt; t += blockDim.x) {
      const float4 d = dirs[t];
      const float c = R.x * d.x + R.y * d.y + R.z * d.z;
      if (c <= 0.f) continue;
      const float kk = ggx_weight(c, alpha) * d.w;
      acc0 += E[3 * t] * kk;
      acc1 += E[3 * t + 1] * kk;
      acc2 += E[3 * t + 2] * kk;
    }
  }
  red[0][threadIdx.x] = acc0;
  red[1][threadIdx.x] = acc1;
  red[2][threadIdx.x] = acc2;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    float* dst = L.out[l] + 3 * k;
    dst[0] = red[0][0] * R.w;
    dst[1] = red[1][0] * R.w;
    dst[2] = red[2][0] * R.w;
  }
}

static LevelSet make_levels(float* const lvl_out[7], const int lh[7], const int lw[7]) {
  LevelSet L;
  L.first[1] = 0;
  for (int l = 0; l < 7; ++l) { L.out[l] = lvl_out ? lvl_out[l] : nullptr; L.h[l] = lh[l]; L.w[l] = lw[l]; }
  for (int l = 1; l <= 6; ++l) L.first[l + 1] = L.first[l] + lh[l] * lw[l];
  return L;
}

hipError_t launch_envmap_out_dirs(int He, int We, const float* in_dirs, const int lh[7],
                                  const int lw[7], float* out_dirs, hipStream_t st) {
  LevelSet L = make_levels(nullptr, lh, lw);
  hipLaunchKernelGGL(envmap_out_dirs_kernel, dim3(L.first[7]), dim3(256), 0, st, He * We,
                     reinterpret_cast<const float4*>(in_dirs), L, reinterpret_cast<float4*>(out_dirs));
  return hipGetLastError();
}

hipError_t launch_envmap_prefilter(const float* E, int He, int We, const float* in_dirs,
                                   const float* out_dirs, float* const lvl_out[7], const int lh[7],
                                   const int lw[7], hipStream_t st) {
  LevelSet L = make_levels(lvl_out, lh, lw);
  hipLaunchKernelGGL(envmap_prefilter_kernel, dim3(L.first[7]), dim3(256), 0, st, E, He * We,
                     reinterpret_cast<const float4*>(in_dirs),
                     reinterpret_cast<const float4*>(out_dirs), L);
  return hipGetLastError();
}

// Adjoint: dE_t = dSpec_0[t] + sum_{l,R} dSpec_l(R) K_l(R,t)/Z_l(R)
//                 + (1/pi) sum_d dIrr(d) max(0, d.d_t) dO_t.
// Thread per input texel; grid.y splits the output texels into chunks whose
// partial sums are added atomically (dE is cleared first; the first chunk adds
// the direct level-0 term).  The output table is read uniformly by the wave.
struct DLevelSet {
  const float* g[7];
  int first[8];
};

__global__ void __launch_bounds__(256) envmap_adjoint_kernel(DLevelSet L, int nt,
                                                             const float4* __restrict__ dirs,
                                                             const float4* __restrict__ out_dirs,
                                                             float* __restrict__ dE, int chunk) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = t < nt;
  const float4 dt = live ? dirs[t] : make_float4(0.f, 0.f, 1.f, 0.f);
  const int o_begin = blockIdx.y * chunk, o_end = min(o_begin + chunk, L.first[7]);
  float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f;
  int l = level_of(L.first, o_begin);
  float alpha = (float)(l * l) / 25.f;
  for (int o = o_begin; o < o_end; ++o) {
    if (o >= L.first[l + 1]) {
      l = level_of(L.first, o);
      alpha = (float)(l * l) / 25.f;
    }
    const float* gg = L.g[l] + 3 * (o - L.first[l]);
    const float g0 = gg[0], g1 = gg[1], g2 = gg[2];
    const float4 R = out_dirs[o];
    const float c = R.x * dt.x + R.y * dt.y + R.z * dt.z;
    if (c <= 0.f) continue;
    const float kk = (l == 6 ? c : ggx_weight(c, alpha)) * dt.w * R.w;
    acc0 += g0 * kk;
    acc1 += g1 * kk;
    acc2 += g2 * kk;
  }
  if (!live) return;
  if (blockIdx.y == 0) {
    acc0 += L.g[0][3 * t];
    acc1 += L.g[0][3 * t + 1];
    acc2 += L.g[0][3 * t + 2];
  }
  atomicAdd(dE + 3 * t, acc0);
  atomicAdd(dE + 3 * t + 1, acc1);
  atomicAdd(dE + 3 * t + 2, acc2);
}

hipError_t launch_envmap_adjoint(const float* const dlvl[7], const int lh[7], const int lw[7],
                                 const float* out_dirs, int He, int We, const float* in_dirs,
                                 float* dE, hipStream_t st) {
  DLevelSet L;
  L.first[1] = 0;
  for (int l = 0; l < 7; ++l) L.g[l] = dlvl[l];
  for (int l = 1; l <= 6; ++l) L.first[l + 1] = L.first[l] + lh[l] * lw[l];
  const int nt = He * We;
  hipError_t e = launch_fill_f32(dE, 0.f, (long long)nt * 3, st);
  if (e != hipSuccess) return e;
  const int chunk = 256;
  const int nchunk = (L.first[7] + chunk - 1) / chunk;
  hipLaunchKernelGGL(envmap_adjoint_kernel, dim3((nt + 255) / 256, nchunk), dim3(256), 0, st, L, nt,
                     reinterpret_cast<const float4*>(in_dirs),
                     reinterpret_cast<const float4*>(out_dirs), dE, chunk);
  return hipGetLastError();
}

// ---------------------------------------------------------------- BRDF table
// Computed once per table in FP64 (the grazing, low-roughness corner of the
// integrand loses several digits in FP32) and rounded to FP32.
__device__ inline double radical_inverse2(uint32_t k) {
  return (double)__builtin_bitreverse32(k) * (1.0 / 4294967296.0);
}

// (beta1, beta2) at vertex (i, j): r = i/(n_r-1), alpha = r^2, n.v =
// max(j/(n_nv-1), 1e-3); GGX half-vector samples from Hammersley points
// ((k + 1/2)/M, radical inverse of k); l = reflect(v, h); weight
// G1(v) G1(l) (v.h)/((n.h)(n.v)) with separable Smith G1 and Schlick Fc.
__global__ void brdf_lut_kernel(float* lut, int n_nv, int n_r, int M) {
  int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n_nv * n_r) return;
  int i = id / n_nv, j = id % n_nv;
  double r = (double)i / (double)(n_r - 1), alpha = r * r, a2 = alpha * alpha;
  double nv = fmax((double)j / (double)(n_nv - 1), 1e-3);
  double vx = sqrt(fmax(0.0, 1.0 - nv * nv)), vz = nv;
  double g1v = 2.0 * nv / (nv + sqrt(a2 + (1.0 - a2) * nv * nv));
  double A = 0.0, B = 0.0;
  for (int k = 0; k < M; ++k) {
    double xi1 = ((double)k + 0.5) / (double)M, xi2 = radical_inverse2((uint32_t)k);
    double ct = sqrt((1.0 - xi1) / (1.0 + (a2 - 1.0) * xi1));
    double stt = sqrt(fmax(0.0, 1.0 - ct * ct));
    double sp, cp;
    sincos(2.0 * 3.14159265358979323846 * xi2, &sp, &cp);
    double hx = stt * cp, hz = ct;
    double vh = vx * hx + vz * hz;
    double lz = 2.0 * vh * hz - vz;
    if (lz <= 0.0) continue;
    double g1l = 2.0 * lz / (lz + sqrt(a2 + (1.0 - a2) * lz * lz));
    double gvis = g1v * g1l * vh / (hz * nv);
    double om = 1.0 - vh;
    double om2 = om * om;
    double fc = om2 * om2 * om;
    A += (1.0 - fc) * gvis;
    B += fc * gvis;
  }
  lut[2 * id] = (float)(A / (double)M);
  lut[2 * id + 1] = (float)(B / (double)M);
}

hipError_t launch_brdf_lut(float* lut, int n_nv, int n_r, int samples, hipStream_t st) {
  int n = n_nv * n_r;
  hipLaunchKernelGGL(brdf_lut_kernel, dim3((n + 127) / 128), dim3(128), 0, st, lut, n_nv, n_r, samples);
  return hipGetLastError();
}

}  // namespace ss
