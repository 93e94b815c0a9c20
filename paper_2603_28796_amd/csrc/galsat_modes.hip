// Straight-through Gumbel training mode and the hand-off kernels
// (candidate pool, confidence, selection) for gfx950.
#include "galsat_device.h"

namespace galsat {

// ------------------------------------------- straight-through Gumbel mode
//
// Two logits per (variable, restart) go through a temperature softmax after
// Gumbel(0,1) noise (Section 3.2, Eq. 3); the forward uses the hard argmax
// (Eq. 4) and the backward the soft probabilities.  With two states only the
// logit difference d = theta1 - theta0 and the noise difference
// l = g1 - g0 matter: y1 = sigma((d + l) / tau), x_hat = [d + l > 0].

// Noise difference of step t for (v, r).  The difference of two
// independent Gumbel(0,1) draws is standard logistic, so it is drawn
// directly by the logistic quantile function from one uniform:
// l = log(u / (1 - u)), u = ((h >> 40) + 0.5) * 2^-24, h the SplitMix64 mix
// of (seed, v * 2^32 + r, t); evaluated in FP64 and rounded once.
__device__ __forceinline__ float gumbel_diff(uint64_t seed, int t, int64_t v, int r) {
  const uint64_t ts = splitmix_mix((uint64_t)(uint32_t)t + 0x632be59bd9b4e019ULL);
  const uint64_t c = ((uint64_t)(uint32_t)v << 32) + (uint64_t)(uint32_t)r;
  const uint64_t h = splitmix_mix(seed ^ splitmix_mix(c ^ ts));
  const double u = ((double)(h >> 40) + 0.5) * (1.0 / 16777216.0);
  return (float)log(u / (1.0 - u));
}

__global__ __launch_bounds__(256) void k_gumbel_noise(float* out, int32_t ldo, int32_t n, int32_t R,
                                                      uint64_t seed, int32_t t) {
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int r = blockIdx.y * 64 + lane;
  if (r >= R) return;
  for (int64_t v = (int64_t)blockIdx.x * 4 + w; v < n; v += (int64_t)gridDim.x * 4)
    out[v * ldo + r] = gumbel_diff(seed, t, v, r);
}

// Hard point of the step: xh = [d + l > 0] (FP32 sum; a tie goes to state
// 0), keeping l for the update.  noise: caller-given l or null to draw it.
__global__ __launch_bounds__(256) void k_gumbel_prep(const float* d, int32_t ldd, const float* noise,
                                                     int32_t ldn, uint64_t seed, int32_t t,
                                                     int32_t n, int32_t R, float* xh, float* nb,
                                                     int32_t ld) {
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int r = blockIdx.y * 64 + lane;
  if (r >= R) return;
  for (int64_t v = (int64_t)blockIdx.x * 4 + w; v < n; v += (int64_t)gridDim.x * 4) {
    const float l = noise ? noise[v * ldn + r] : gumbel_diff(seed, t, v, r);
    const float s = d[v * ldd + r] + l;
    xh[v * ld + r] = s > 0.0f ? 1.0f : 0.0f;
    nb[v * ld + r] = l;
  }
}

// Soft backward and update: g1 = G * y1 (1 - y1) / tau reaches theta1 and
// -g1 reaches theta0, so d moves by twice theta1's step (SGD, or Adam whose
// theta0 moments are the exact negatives of theta1's).
__global__ __launch_bounds__(256) void k_gumbel_update(float* d, int32_t ldd, const float* nb,
                                                       const float* G, int32_t ld, float* mom,
                                                       float* vel, int32_t ldm, int32_t n,
                                                       int32_t R, float tau, float lr, float b1,
                                                       float b2, float eps, double inv_c1,
                                                       double inv_c2, int32_t adam) {
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int r = blockIdx.y * 64 + lane;
  if (r >= R) return;
  for (int64_t v = (int64_t)blockIdx.x * 4 + w; v < n; v += (int64_t)gridDim.x * 4) {
    const double dv = d[v * ldd + r];
    const double z = (dv + (double)nb[v * ld + r]) / (double)tau;
    const double y1 = 1.0 / (1.0 + exp(-z));
    const double g1 = (double)G[v * ld + r] * y1 * (1.0 - y1) / (double)tau;
    double step;
    if (adam) {
      const double mm = (double)b1 * (double)mom[v * ldm + r] + (1.0 - (double)b1) * g1;
      const double vv = (double)b2 * (double)vel[v * ldm + r] + (1.0 - (double)b2) * g1 * g1;
      mom[v * ldm + r] = (float)mm;
      vel[v * ldm + r] = (float)vv;
      step = (double)lr * ((double)(float)mm * inv_c1) /
             (sqrt((double)(float)vv * inv_c2) + (double)eps);
    } else {
      step = (double)lr * g1;
    }
    d[v * ldd + r] = (float)(dv - 2.0 * step);
  }
}

// ---------------------------------------------------------- hand-off
//
// Candidate pool of Section 3.3.1, Eq. (8): candidate k of formula f adds
// the noise difference of "step" k, restart 0 to the logit difference of
// f's selected restart and takes the argmax; its confidence is the
// perturbed probability of the value taken.
__global__ __launch_bounds__(256) void k_candidates(const float* d, int32_t ldd,
                                                    const int32_t* var_formula, const int32_t* best,
                                                    int32_t n, uint64_t seed, float tau,
                                                    uint8_t* assign, float* conf) {
  const int k = blockIdx.y;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int r = best[var_formula[v]];
    const float dv = d[v * ldd + r];
    const float l = gumbel_diff(seed, k, v, 0);
    const bool one = dv + l > 0.0f;
    const double y1 = 1.0 / (1.0 + exp(-((double)dv + (double)l) / (double)tau));
    assign[(int64_t)k * n + v] = one ? 1 : 0;
    conf[(int64_t)k * n + v] = (float)(one ? y1 : 1.0 - y1);
  }
}

// Unperturbed confidence max(p, 1 - p), p = sigma(d / tau), of each
// variable at its formula's selected restart (Section 3.3.2).
__global__ __launch_bounds__(256) void k_confidence(const float* d, int32_t ldd,
                                                    const int32_t* var_formula, const int32_t* best,
                                                    int32_t n, float tau, float* conf) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const double p = 1.0 / (1.0 + exp(-(double)d[v * ldd + best[var_formula[v]]] / (double)tau));
    conf[v] = (float)(p > 0.5 ? p : 1.0 - p);
  }
}

// Selection of the S_f most (HIGH) or least confident variables of formula
// f in candidate k, ties to the lower index, written in increasing index
// order.  Keys are 64-bit: confidence bits (inverted for LOW) above the
// inverted local index, so every key is distinct and larger = preferred.
// An exact radix select (8-bit digits from the top, integer counts in LDS)
// finds the S-th largest key; a block scan then compacts the selected
// indices.
template <bool HIGH>
__device__ __forceinline__ uint64_t sel_key(float c, int local) {
  const uint32_t b = __float_as_uint(c);
  const uint64_t hi = HIGH ? b : ~b;
  return (hi << 32) | (uint64_t)(~(uint32_t)local);
}

// Adds one to hist[bin] for every active lane.  Confidences share their top
// key bytes, so most lanes of a wave usually name the same bin: the lanes
// that share the first active lane's bin add their count with one atomic,
// the rest add one each.
__device__ __forceinline__ void hist_add(uint32_t* hist, bool act, uint32_t bin) {
  const uint64_t am = __ballot(act);
  if (am == 0) return;
  const int lead = __builtin_ctzll(am);
  const uint32_t lb = (uint32_t)__shfl((int)bin, lead, 64);
  const bool same = act && bin == lb;
  const uint64_t sm = __ballot(same);
  if ((int)(threadIdx.x & 63) == lead) atomicAdd(&hist[lb], (uint32_t)__popcll(sm));
  if (act && !same) atomicAdd(&hist[bin], 1u);
}

constexpr int kSelU = 8;  // confidence loads in flight per thread

template <bool HIGH>
__global__ __launch_bounds__(1024) void k_select(const float* conf, int32_t n,
                                                 const int32_t* f_vbeg, const int32_t* sel_off,
                                                 int32_t stot, int32_t* out) {
  const int f = blockIdx.x, k = blockIdx.y, tid = threadIdx.x, nt = blockDim.x;
  const int v0 = f_vbeg[f], nf = f_vbeg[f + 1] - v0;
  const int S = sel_off[f + 1] - sel_off[f];
  if (S <= 0) return;
  const float* c = conf + (int64_t)k * n + v0;
  __shared__ uint32_t hist[256];
  __shared__ uint64_t s_prefix, s_mask;
  __shared__ int s_rank, s_done;
  if (tid == 0) {
    s_prefix = 0;
    s_mask = 0;
    s_rank = S;
    s_done = 0;
  }
  __syncthreads();
  for (int pass = 0; pass < 8; ++pass) {
    const int shift = 56 - 8 * pass;
    for (int b = tid; b < 256; b += nt) hist[b] = 0;
    __syncthreads();
    const uint64_t prefix = s_prefix, mask = s_mask;
    // kSelU block strides per iteration, all their loads issued first; the
    // loop runs the same count on every lane, so the ballots see whole waves
    for (int base = 0; base < nf; base += nt * kSelU) {
      float cv[kSelU];
#pragma unroll
      for (int u = 0; u < kSelU; ++u) {
        const int i = base + u * nt + tid;
        cv[u] = i < nf ? c[i] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < kSelU; ++u) {
        const int i = base + u * nt + tid;
        const uint64_t key = sel_key<HIGH>(cv[u], i);
        hist_add(hist, i < nf && (key & mask) == prefix, (uint32_t)(key >> shift) & 255u);
      }
    }
    __syncthreads();
    if (tid == 0) {
      int rank = s_rank, acc = 0, chosen = 0;
      for (int b = 255; b >= 0; --b) {
        if (acc + (int)hist[b] >= rank) {
          chosen = b;
          rank -= acc;
          break;
        }
        acc += (int)hist[b];
      }
      s_prefix = prefix | ((uint64_t)chosen << shift);
      s_mask = mask | (0xFFULL << shift);
      s_rank = rank;
      // every key under the new prefix is selected: keys >= the prefix with
      // zero lower digits are exactly the selection
      s_done = (int)hist[chosen] == rank;
    }
    __syncthreads();
    if (s_done) break;
  }
  const uint64_t thr = s_prefix;  // keys >= thr are the selection
  // exclusive scan of the per-thread counts: within each wave by shuffles,
  // then over the wave totals
  __shared__ int wave_tot[16];
  const int per = (nf + nt - 1) / nt;
  const int i0 = tid * per, i1 = min(nf, i0 + per);
  // each thread's contiguous run, kSelU loads in flight (indices clamped
  // into the run, the extra entries not counted)
  int mine = 0;
  for (int i = i0; i < i1; i += kSelU) {
    float cv[kSelU];
#pragma unroll
    for (int u = 0; u < kSelU; ++u) cv[u] = c[min(i + u, i1 - 1)];
#pragma unroll
    for (int u = 0; u < kSelU; ++u) mine += (i + u < i1 && sel_key<HIGH>(cv[u], i + u) >= thr) ? 1 : 0;
  }
  const int lane = tid & 63, w = tid >> 6;
  int incl = mine;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) wave_tot[w] = incl;
  __syncthreads();
  int pos = incl - mine;
  for (int u = 0; u < w; ++u) pos += wave_tot[u];
  int32_t* o = out + (int64_t)k * stot + sel_off[f];
  for (int i = i0; i < i1; i += kSelU) {
    float cv[kSelU];
#pragma unroll
    for (int u = 0; u < kSelU; ++u) cv[u] = c[min(i + u, i1 - 1)];
#pragma unroll
    for (int u = 0; u < kSelU; ++u)
      if (i + u < i1 && sel_key<HIGH>(cv[u], i + u) >= thr) o[pos++] = v0 + i + u;
  }
}

// ------------------------------------------------------------ launchers

hipError_t launch_gumbel_noise(float* out, int32_t ldo, int32_t n, int32_t R, uint64_t seed,
                               int32_t t, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  dim3 grid(grid_x_for(((int64_t)n + 3) / 4), (R + 63) / 64), block(256);
  hipLaunchKernelGGL(k_gumbel_noise, grid, block, 0, s, out, ldo, n, R, seed, t);
  return hipGetLastError();
}

hipError_t launch_gumbel_prep(const float* d, int32_t ldd, const float* noise, int32_t ldn,
                              uint64_t seed, int32_t t, int32_t n, int32_t R, float* xh, float* nb,
                              int32_t ld, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  dim3 grid(grid_x_for(((int64_t)n + 3) / 4), (R + 63) / 64), block(256);
  hipLaunchKernelGGL(k_gumbel_prep, grid, block, 0, s, d, ldd, noise, ldn, seed, t, n, R, xh, nb, ld);
  return hipGetLastError();
}

hipError_t launch_gumbel_update(float* d, int32_t ldd, const float* nb, const float* G, int32_t ld,
                                float* mom, float* vel, int32_t ldm, int32_t n, int32_t R, float tau,
                                float lr, float b1, float b2, float eps, double inv_c1,
                                double inv_c2, int32_t adam, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  dim3 grid(grid_x_for(((int64_t)n + 3) / 4), (R + 63) / 64), block(256);
  hipLaunchKernelGGL(k_gumbel_update, grid, block, 0, s, d, ldd, nb, G, ld, mom, vel, ldm, n, R, tau,
                     lr, b1, b2, eps, inv_c1, inv_c2, adam);
  return hipGetLastError();
}

hipError_t launch_candidates(const float* d, int32_t ldd, const int32_t* var_formula,
                             const int32_t* best, int32_t n, int32_t num, uint64_t seed, float tau,
                             uint8_t* assign, float* conf, hipStream_t s) {
  if (n <= 0 || num <= 0) return hipSuccess;
  dim3 grid(grid_x_for(((int64_t)n + 255) / 256), num), block(256);
  hipLaunchKernelGGL(k_candidates, grid, block, 0, s, d, ldd, var_formula, best, n, seed, tau, assign,
                     conf);
  return hipGetLastError();
}

hipError_t launch_confidence(const float* d, int32_t ldd, const int32_t* var_formula,
                             const int32_t* best, int32_t n, float tau, float* conf, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_confidence, dim3(grid_x_for(((int64_t)n + 255) / 256)), dim3(256), 0, s, d,
                     ldd, var_formula, best, n, tau, conf);
  return hipGetLastError();
}

hipError_t launch_select(const float* conf, int32_t n, int32_t F, const int32_t* f_vbeg,
                         const int32_t* sel_off, int32_t stot, int32_t num, bool highest,
                         int32_t* out, hipStream_t s) {
  if (F <= 0 || num <= 0 || stot <= 0) return hipSuccess;
  dim3 grid(F, num), block(1024);
  if (highest)
    hipLaunchKernelGGL((k_select<true>), grid, block, 0, s, conf, n, f_vbeg, sel_off, stot, out);
  else
    hipLaunchKernelGGL((k_select<false>), grid, block, 0, s, conf, n, f_vbeg, sel_off, stot, out);
  return hipGetLastError();
}

}  // namespace galsat
