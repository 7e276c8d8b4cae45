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

// D(mu; alpha) c with mu^2 = (1 + c)/2 (hardware reciprocal: the weights enter
// normalised sums).  With k = (alpha^2 - 1)/2 the denominator
// t = 1 + mu^2 (alpha^2 - 1) is one fused multiply-add, c k + (k + 1);
// ggx_scaled leaves out the factor alpha^2 / pi.
__device__ __forceinline__ float ggx_scaled(float c, float k) {
  const float t = __builtin_fmaf(c, k, k + 1.f);
  return __builtin_amdgcn_rcpf(t * t) * c;
}
__device__ inline float ggx_weight(float c, float alpha) {
  const float a2 = alpha * alpha;
  return a2 * (1.f / kPi) * ggx_scaled(c, 0.5f * (a2 - 1.f));
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

// Prefilter, stage 1.  Block (x, y): 512 consecutive output texels of levels
// 1..6 (two per thread) against input chunk y.  The chunk's texels are staged
// through LDS 256 at a time (every thread then reads the same entry: a
// broadcast), so each input texel is fetched once per 512 outputs instead of
// once per output.  A staged batch whose latitude band lies beyond the
// hemisphere of every output direction of the wave (angular distance above
// pi/2 + 1e-3, so the cosine is clearly negative in FP32) adds nothing and is
// skipped.  Partial sums go to part[y][o][3]; stage 2 adds the chunks in a
// fixed order.
__global__ void __launch_bounds__(256) envmap_prefilter_kernel(const float* __restrict__ E, int He, int We,
                                                               int chunk, const float4* __restrict__ dirs,
                                                               const float4* __restrict__ out_dirs,
                                                               int n_out, LevelSet L, float* __restrict__ part) {
  __shared__ float4 sd[256];
  __shared__ float4 se[256];  // (E, -): one 16-byte broadcast read per input texel
  const int nt = He * We;
  // two output texels per thread, 256 apart, so that each staged input texel
  // read from LDS serves two of them
  const int oA = blockIdx.x * 512 + threadIdx.x, oB = oA + 256;
  const bool liveA = oA < n_out, liveB = oB < n_out;
  const int ooA = liveA ? oA : n_out - 1, ooB = liveB ? oB : n_out - 1;
  const int lA = level_of(L.first, ooA), lB = level_of(L.first, ooB);
  const float4 RA = out_dirs[ooA], RB = out_dirs[ooB];
  const float alA = (float)(lA * lA) / 25.f, alB = (float)(lB * lB) / 25.f;
  const float thA = acosf(fminf(fmaxf(RA.z, -1.f), 1.f)), thB = acosf(fminf(fmaxf(RB.z, -1.f), 1.f));
  const int t0 = blockIdx.y * chunk, t1 = min(t0 + chunk, nt);
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, b0 = 0.f, b1 = 0.f, b2 = 0.f;
  for (int tb = t0; tb < t1; tb += 256) {
    const int n = min(256, t1 - tb);
    // latitude band of the batch (texel-centre angles of its first and last rows)
    const float tha = kPi * ((float)(tb / We) + 0.5f) / (float)He;
    const float thb = kPi * ((float)((tb + n - 1) / We) + 0.5f) / (float)He;
    const float gapA = fmaxf(fmaxf(tha - thA, thA - thb), 0.f), gapB = fmaxf(fmaxf(tha - thB, thB - thb), 0.f);
    const bool skip = __ballot(!(gapA > 0.5f * kPi + 1e-3f) || !(gapB > 0.5f * kPi + 1e-3f)) == 0ull;
    __syncthreads();
    if (threadIdx.x < n) {
      const int t = tb + threadIdx.x;
      sd[threadIdx.x] = dirs[t];
      se[threadIdx.x] = make_float4(E[3 * t], E[3 * t + 1], E[3 * t + 2], 0.f);
    }
    __syncthreads();
    if (skip) continue;
    // texels behind an output direction (c <= 0) get weight exactly 0 through
    // max(c, 0) (both weights carry a factor c), with no select or branch:
    // lanes of a wave face different ways, and a branch let the compiler sink
    // part of the staged reads into it and wait for LDS once per texel
    if (lA == 6 && lB == 6) {
#pragma unroll 4
      for (int i = 0; i < n; ++i) {
        const float4 d = sd[i], e = se[i];
        const float cA = fmaxf(RA.x * d.x + RA.y * d.y + RA.z * d.z, 0.f);
        const float cB = fmaxf(RB.x * d.x + RB.y * d.y + RB.z * d.z, 0.f);
        const float kA = cA * d.w, kB = cB * d.w;
        a0 += e.x * kA; a1 += e.y * kA; a2 += e.z * kA;
        b0 += e.x * kB; b1 += e.y * kB; b2 += e.z * kB;
      }
    } else if (lA < 6 && lB < 6) {
#pragma unroll 4
      for (int i = 0; i < n; ++i) {
        const float4 d = sd[i], e = se[i];
        const float cA = fmaxf(RA.x * d.x + RA.y * d.y + RA.z * d.z, 0.f);
        const float cB = fmaxf(RB.x * d.x + RB.y * d.y + RB.z * d.z, 0.f);
        const float kA = ggx_weight(cA, alA) * d.w, kB = ggx_weight(cB, alB) * d.w;
        a0 += e.x * kA; a1 += e.y * kA; a2 += e.z * kA;
        b0 += e.x * kB; b1 += e.y * kB; b2 += e.z * kB;
      }
    } else {
      // a thread whose two texels straddle the last specular level and the
      // irradiance level
      for (int i = 0; i < n; ++i) {
        const float4 d = sd[i], e = se[i];
        const float cA = fmaxf(RA.x * d.x + RA.y * d.y + RA.z * d.z, 0.f);
        const float cB = fmaxf(RB.x * d.x + RB.y * d.y + RB.z * d.z, 0.f);
        const float kA = (lA == 6 ? cA : ggx_weight(cA, alA)) * d.w;
        const float kB = (lB == 6 ? cB : ggx_weight(cB, alB)) * d.w;
        a0 += e.x * kA; a1 += e.y * kA; a2 += e.z * kA;
        b0 += e.x * kB; b1 += e.y * kB; b2 += e.z * kB;
      }
    }
  }
  if (liveA) {
    float* dst = part + ((long long)blockIdx.y * n_out + oA) * 3;
    dst[0] = a0;
    dst[1] = a1;
    dst[2] = a2;
  }
  if (liveB) {
    float* dst = part + ((long long)blockIdx.y * n_out + oB) * 3;
    dst[0] = b0;
    dst[1] = b1;
    dst[2] = b2;
  }
}

// Prefilter, stage 2: level texel = (sum over chunks) / Z.
__global__ void __launch_bounds__(256) envmap_prefilter_sum_kernel(const float* __restrict__ part, int n_chunks,
                                                                   int n_out, const float4* __restrict__ out_dirs,
                                                                   LevelSet L) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n_out) return;
  float a0 = 0.f, a1 = 0.f, a2 = 0.f;
  for (int y = 0; y < n_chunks; ++y) {
    const float* p = part + ((long long)y * n_out + o) * 3;
    a0 += p[0];
    a1 += p[1];
    a2 += p[2];
  }
  const int l = level_of(L.first, o);
  const float iz = out_dirs[o].w;
  float* dst = L.out[l] + 3 * (o - L.first[l]);
  dst[0] = a0 * iz;
  dst[1] = a1 * iz;
  dst[2] = a2 * iz;
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

int envmap_prefilter_chunks(int He, int We) {
  // input chunks of at least 512 texels: a 128 x 256 map gives 64 chunks, so
  // the launch has about 13 waves per SIMD to hide its staging barriers
  const int nt = He * We;
  int c = (nt + 511) / 512;
  return c < 1 ? 1 : (c > kEnvChunksMax ? kEnvChunksMax : c);
}

hipError_t launch_envmap_prefilter(const float* E, int He, int We, const float* in_dirs,
                                   const float* out_dirs, float* const lvl_out[7], const int lh[7],
                                   const int lw[7], float* part, hipStream_t st) {
  LevelSet L = make_levels(lvl_out, lh, lw);
  const int n_out = L.first[7], nt = He * We;
  const int nc = envmap_prefilter_chunks(He, We);
  const int chunk = ((nt + nc - 1) / nc + 255) / 256 * 256;
  hipLaunchKernelGGL(envmap_prefilter_kernel, dim3((n_out + 511) / 512, nc), dim3(256), 0, st, E, He, We, chunk,
                     reinterpret_cast<const float4*>(in_dirs),
                     reinterpret_cast<const float4*>(out_dirs), n_out, L, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(envmap_prefilter_sum_kernel, dim3((n_out + 255) / 256), dim3(256), 0, st, part, nc, n_out,
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
  int h[7], w[7];
};

__global__ void __launch_bounds__(256) envmap_adjoint_kernel(DLevelSet L, int nt,
                                                             const float4* __restrict__ dirs,
                                                             const float4* __restrict__ out_dirs,
                                                             float* __restrict__ dE, int chunk,
                                                             float* __restrict__ part) {
  __shared__ float4 sR[256], sG[256];
  // two input texels per thread, 256 apart, so that each staged output texel
  // read from LDS serves two evaluations
  const int t0 = blockIdx.x * 512 + threadIdx.x, t1 = t0 + 256;
  const bool live0 = t0 < nt, live1 = t1 < nt;
  const float4 d0 = live0 ? dirs[t0] : make_float4(0.f, 0.f, 1.f, 0.f);
  const float4 d1 = live1 ? dirs[t1] : make_float4(0.f, 0.f, 1.f, 0.f);
  const int o_begin = blockIdx.y * chunk, o_end = min(o_begin + chunk, L.first[7]);
  // Latitude bands of the block's input texels and of the chunk's output texels
  // (texel-centre angles; rows are monotone within a level).  When they are
  // more than pi/2 + 1e-3 apart every cosine is clearly negative and the chunk
  // adds nothing.
  bool skip;
  {
    const int He = L.h[0], We = L.w[0];
    const int ta = blockIdx.x * 512, tb = min(ta + 512, nt) - 1;
    const float ia = kPi * ((float)(ta / We) + 0.5f) / (float)He, ib = kPi * ((float)(tb / We) + 0.5f) / (float)He;
    float oa = 4.f, ob = -1.f;
    for (int lv = level_of(L.first, o_begin); lv <= 6 && L.first[lv] < o_end; ++lv) {
      const int k0 = max(o_begin, L.first[lv]) - L.first[lv], k1 = min(o_end, L.first[lv + 1]) - 1 - L.first[lv];
      oa = fminf(oa, kPi * ((float)(k0 / L.w[lv]) + 0.5f) / (float)L.h[lv]);
      ob = fmaxf(ob, kPi * ((float)(k1 / L.w[lv]) + 0.5f) / (float)L.h[lv]);
    }
    skip = fmaxf(ia - ob, oa - ib) > 0.5f * kPi + 1e-3f;
  }
  // Stage the chunk's output texels through LDS (direction and 1/Z; gradient
  // and the GGX constant); the loops below then read them as broadcasts, four
  // texels' reads issued together, instead of a chain of dependent scalar
  // loads per output texel.
  if (!skip) {
    const int o = o_begin + (int)threadIdx.x;
    if (o < o_end) {
      const int l = level_of(L.first, o);
      const float* gg = L.g[l] + 3 * (o - L.first[l]);
      // specular levels: k = (alpha^2 - 1)/2 in w, and alpha^2 / pi folded into 1/Z
      const float alpha = (float)(l * l) / 25.f, a2 = alpha * alpha;
      float4 R = out_dirs[o];
      if (l < 6) R.w *= a2 * (1.f / kPi);
      sR[threadIdx.x] = R;
      sG[threadIdx.x] = make_float4(gg[0], gg[1], gg[2], 0.5f * (a2 - 1.f));
    }
  }
  __syncthreads();
  float a00 = 0.f, a01 = 0.f, a02 = 0.f, a10 = 0.f, a11 = 0.f, a12 = 0.f;
  if (!skip) {
    // the specular levels come first in the flattened output order, the
    // irradiance level last; weights are exactly 0 for c <= 0 through max(c, 0)
    // (both carry a factor c), without a branch
    const int n = o_end - o_begin, i6 = min(max(L.first[6] - o_begin, 0), n);
#pragma unroll 4
    for (int i = 0; i < i6; ++i) {
      const float4 R = sR[i], G = sG[i];
      const float c0 = fmaxf(R.x * d0.x + R.y * d0.y + R.z * d0.z, 0.f);
      const float c1 = fmaxf(R.x * d1.x + R.y * d1.y + R.z * d1.z, 0.f);
      const float k0 = ggx_scaled(c0, G.w) * d0.w * R.w, k1 = ggx_scaled(c1, G.w) * d1.w * R.w;
      a00 += G.x * k0; a01 += G.y * k0; a02 += G.z * k0;
      a10 += G.x * k1; a11 += G.y * k1; a12 += G.z * k1;
    }
#pragma unroll 4
    for (int i = i6; i < n; ++i) {
      const float4 R = sR[i], G = sG[i];
      const float c0 = fmaxf(R.x * d0.x + R.y * d0.y + R.z * d0.z, 0.f);
      const float c1 = fmaxf(R.x * d1.x + R.y * d1.y + R.z * d1.z, 0.f);
      const float k0 = c0 * d0.w * R.w, k1 = c1 * d1.w * R.w;
      a00 += G.x * k0; a01 += G.y * k0; a02 += G.z * k0;
      a10 += G.x * k1; a11 += G.y * k1; a12 += G.z * k1;
    }
  }
  // each texel's sums: the first chunk adds the direct level-0 term; then the
  // chunk's partials (deterministic, added in chunk order afterwards) or atomics
  auto put = [&](int t, float acc0, float acc1, float acc2) {
    if (blockIdx.y == 0) {
      acc0 += L.g[0][3 * t];
      acc1 += L.g[0][3 * t + 1];
      acc2 += L.g[0][3 * t + 2];
    }
    if (part) {
      float* p = part + ((long long)blockIdx.y * nt + t) * 3;
      p[0] = acc0;
      p[1] = acc1;
      p[2] = acc2;
      return;
    }
    atomicAdd(dE + 3 * t, acc0);
    atomicAdd(dE + 3 * t + 1, acc1);
    atomicAdd(dE + 3 * t + 2, acc2);
  };
  if (live0) put(t0, a00, a01, a02);
  if (live1) put(t1, a10, a11, a12);
}

__global__ void envmap_adjoint_reduce_kernel(const float* __restrict__ part, int n, int nchunk, float* __restrict__ dE) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float acc = 0.f;
  for (int c = 0; c < nchunk; ++c) acc += part[(long long)c * n + i];
  dE[i] = acc;
}

int envmap_adjoint_chunks(int lh_total) { return (lh_total + 255) / 256; }

hipError_t launch_envmap_adjoint(const float* const dlvl[7], const int lh[7], const int lw[7],
                                 const float* out_dirs, int He, int We, const float* in_dirs,
                                 float* dE, const int* status, float* part, hipStream_t st) {
  DLevelSet L;
  L.first[1] = 0;
  for (int l = 0; l < 7; ++l) L.g[l] = dlvl[l];
  for (int l = 1; l <= 6; ++l) L.first[l + 1] = L.first[l] + lh[l] * lw[l];
  for (int l = 0; l < 7; ++l) { L.h[l] = lh[l]; L.w[l] = lw[l]; }
  L.h[0] = He; L.w[0] = We;
  const int nt = He * We;
  hipError_t e = launch_fill_f32(dE, 0.f, (long long)nt * 3, st);
  if (e != hipSuccess) return e;
  const int chunk = 256;
  const int nchunk = (L.first[7] + chunk - 1) / chunk;
  hipLaunchKernelGGL(envmap_adjoint_kernel, dim3((nt + 511) / 512, nchunk), dim3(256), 0, st, L, nt,
                     reinterpret_cast<const float4*>(in_dirs),
                     reinterpret_cast<const float4*>(out_dirs), dE, chunk, part);
  e = hipGetLastError();
  if (e == hipSuccess && part)
    hipLaunchKernelGGL(envmap_adjoint_reduce_kernel, dim3((3 * nt + 255) / 256), dim3(256), 0, st, part, 3 * nt,
                       nchunk, dE);
  e = hipGetLastError();
  if (e != hipSuccess || !status) return e;
  return launch_poison_if_capacity(dE, (long long)nt * 3, status, st);
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
