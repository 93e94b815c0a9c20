// Persistent LDS schedule (gfx950): for formulas small enough that a
// restart group's state fits in LDS, one workgroup per (formula, restart
// group) runs every step of galsat_step in one launch.  The state is
// double-buffered in LDS (every variable updates from the same x_k:
// Jacobi); the formula's occurrence records and var_ptr slice are copied
// to LDS once per launch when they fit (else read from global memory), so
// a step touches global memory only for its trace entries.  Each step's
// loss' and rounded unsat count are reduced in a fixed order (wave
// butterflies, then the waves in index order).  The gradient of a variable
// is summed over its occurrences in var_occ order in FP64 from the same
// FP32 products as the variable pass (Section 3.2, Eq. 2 and its
// derivative), so states equal the general schedule's bitwise when no
// variable is split.
#include "galsat_device.h"

namespace galsat {

namespace {

constexpr int kPersistWaves = kPersistBlock / 64;

struct PersistLayout {
  size_t occ, red_l, red_u, vp, x, total;
};

// byte offsets of the dynamic LDS areas; records first (16-byte aligned)
__host__ __device__ inline PersistLayout persist_layout(int rg, int nf_max, int nocc_stage) {
  PersistLayout p;
  p.occ = 0;
  p.red_l = p.occ + (size_t)nocc_stage * 16;                           // double [2][waves][rg]
  p.red_u = p.red_l + (size_t)2 * kPersistWaves * rg * sizeof(double); // int [2][waves][rg]
  p.vp = p.red_u + (size_t)2 * kPersistWaves * rg * sizeof(int);      // int [nf_max + 1]
  p.x = p.vp + (((size_t)nf_max + 1) * sizeof(int) + 15) / 16 * 16;    // float [2][nf_max][rg]
  p.total = p.x + (size_t)2 * nf_max * rg * sizeof(float);
  return p;
}

template <int RG>
__device__ __forceinline__ float lds_row(const float* xs, int vb, int code, int lane) {
  return xs[((code >> 1) - vb) * RG + lane];
}

// STAGED picks where the records are read (LDS or global memory) at compile
// time, so that every load has one address space (no generic loads).
template <int RG, bool STAGED>
__global__ __launch_bounds__(kPersistBlock) void k_persistent(PersistArgs a) {
  constexpr int IPB = kPersistBlock / RG;
  extern __shared__ int4 smem4[];
  char* smem = reinterpret_cast<char*>(smem4);
  const PersistLayout lay = persist_layout(RG, a.nf_max, STAGED ? a.nocc_max : 0);
  int4* s_occ = reinterpret_cast<int4*>(smem + lay.occ);
  double* s_l = reinterpret_cast<double*>(smem + lay.red_l);
  int* s_u = reinterpret_cast<int*>(smem + lay.red_u);
  int* s_vp = reinterpret_cast<int*>(smem + lay.vp);
  float* xa = reinterpret_cast<float*>(smem + lay.x);
  float* xb = xa + (int64_t)a.nf_max * RG;
  const int groups = (a.R + RG - 1) / RG;
  const int f = a.f_order[blockIdx.x / groups], grp = blockIdx.x % groups;
  const int lane = threadIdx.x % RG, slot = threadIdx.x / RG;
  const int wave = threadIdx.x / 64, wlane = threadIdx.x % 64;
  const int r = grp * RG + lane;
  const bool active = r < a.R;
  const int vb = a.f_vbeg[f], nf = a.f_vbeg[f + 1] - vb;
  const int qb = a.var_ptr[vb];
  for (int i = threadIdx.x; i <= nf; i += kPersistBlock) s_vp[i] = a.var_ptr[vb + i] - qb;
  if constexpr (STAGED) {
    const int nocc = a.var_ptr[vb + nf] - qb;
    for (int i = threadIdx.x; i < nocc; i += kPersistBlock) s_occ[i] = a.occ[qb + i];
  }
  for (int i = threadIdx.x; i < nf * RG; i += kPersistBlock) {
    const int rr = grp * RG + i % RG;
    xa[i] = rr < a.R ? a.x[(int64_t)(vb + i / RG) * a.ldx + rr] : 0.0f;
  }
  __syncthreads();
  for (int k = 0; k < a.steps; ++k) {
    double lsum = 0.0;
    int usum = 0;
    for (int vi = slot; vi < nf; vi += IPB) {
      const float xv = xa[vi * RG + lane];
      double g = 0.0;
      const int q0 = s_vp[vi], q1 = s_vp[vi + 1];
      // one occurrence's contribution, in var_occ order (q is formula-local)
      auto add = [&](const int4 o, int q) {
        const int hdr = o.x, nother = rec_nother(hdr);
        const bool first = rec_first(hdr), neg = rec_neg(hdr);
        float prod = 1.0f;
        bool any_true = false;
        if (rec_kind(hdr) == kRecInline) {
          int codes[7] = {o.y, o.z, o.w, 0, 0, 0, 0};
          if (nother > 3) {
            const int4 e = a.occx[qb + q];
            codes[3] = e.x; codes[4] = e.y; codes[5] = e.z; codes[6] = e.w;
          }
#pragma unroll
          for (int c = 0; c < 7; ++c) {
            if (c < nother) {
              const float y = lds_row<RG>(xa, vb, codes[c], lane);
              prod *= lit_factor(codes[c], y);
              any_true = any_true || lit_true(codes[c], y);
            }
          }
        } else {  // GENERAL: the clause's other literals in clause order
          const int t = o.y, p = o.z;
          for (int i = a.clause_ptr[t]; i < a.clause_ptr[t + 1]; ++i) {
            if (i == p) continue;
            const int code = a.clause_lits[i];
            const float y = lds_row<RG>(xa, vb, code, lane);
            prod *= lit_factor(code, y);
            any_true = any_true || lit_true(code, y);
          }
        }
        g += (double)(neg ? prod : -prod);
        if (first) {
          const int own = neg ? 1 : 0;
          lsum += (double)(lit_factor(own, xv) * prod);
          usum += (any_true || lit_true(own, xv)) ? 0 : 1;
        }
      };
      // the same contribution for an inline record with at most three other
      // literals whose states are already read (an absent literal's factor
      // is exactly 1, so the product is the same)
      auto add3 = [&](const int4 o, const float* y) {
        const int hdr = o.x, nother = rec_nother(hdr);
        const bool first = rec_first(hdr), neg = rec_neg(hdr);
        const int codes[3] = {o.y, o.z, o.w};
        float prod = 1.0f;
        bool any_true = false;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const bool here = c < nother;
          prod *= here ? lit_factor(codes[c], y[c]) : 1.0f;
          any_true = any_true || (here && lit_true(codes[c], y[c]));
        }
        g += (double)(neg ? prod : -prod);
        if (first) {
          const int own = neg ? 1 : 0;
          lsum += (double)(lit_factor(own, xv) * prod);
          usum += (any_true || lit_true(own, xv)) ? 0 : 1;
        }
      };
      const int4* recs;
      if constexpr (STAGED) recs = s_occ;
      else recs = a.occ + qb;
      const int self = (vb + vi) << 1;  // a code whose state row is in LDS
      // four records in flight; a partial last batch re-reads its last
      // record and masks the extra contributions off
      for (int q = q0; q < q1; q += 4) {
        int4 o[4];
        bool ok[4];
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) {
          ok[k2] = q + k2 < q1;
          o[k2] = recs[ok[k2] ? q + k2 : q1 - 1];
        }
        bool short3 = true;
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2)
          short3 = short3 && rec_kind(o[k2].x) == kRecInline && rec_nother(o[k2].x) <= 3;
        if (short3) {  // every state read of the four issued before any use
          float y[4][3];
#pragma unroll
          for (int k2 = 0; k2 < 4; ++k2) {
            const int nother = rec_nother(o[k2].x);
            y[k2][0] = lds_row<RG>(xa, vb, nother > 0 ? o[k2].y : self, lane);
            y[k2][1] = lds_row<RG>(xa, vb, nother > 1 ? o[k2].z : self, lane);
            y[k2][2] = lds_row<RG>(xa, vb, nother > 2 ? o[k2].w : self, lane);
          }
#pragma unroll
          for (int k2 = 0; k2 < 4; ++k2)
            if (ok[k2]) add3(o[k2], y[k2]);
        } else {
#pragma unroll
          for (int k2 = 0; k2 < 4; ++k2)
            if (ok[k2]) add(o[k2], q + k2);
        }
      }
      xb[vi * RG + lane] = clamp01((double)xv - (double)a.lr * g);
    }
    // fixed-order reduction over the slots of each restart: butterflies over
    // the wave's slots, then the waves in index order; buffers alternate by
    // step so one barrier per step suffices
#pragma unroll
    for (int off = RG; off < 64; off <<= 1) {
      lsum += __shfl_xor(lsum, off);
      usum += __shfl_xor(usum, off);
    }
    const int buf = (k & 1) * kPersistWaves * RG;
    if (wlane < RG) {
      s_l[buf + wave * RG + lane] = lsum;
      s_u[buf + wave * RG + lane] = usum;
    }
    float* tmp = xa;
    xa = xb;
    xb = tmp;
    __syncthreads();
    if (threadIdx.x < RG && active) {
      double tot = 0.0;
      int utot = 0;
#pragma unroll
      for (int w = 0; w < kPersistWaves; ++w) {
        tot += s_l[buf + w * RG + lane];
        utot += s_u[buf + w * RG + lane];
      }
      const int64_t o = ((int64_t)k * a.F + f) * a.R + r;
      if (a.loss_trace) a.loss_trace[o] = (float)(tot + (double)a.n_empty[f]);
      if (a.unsat_trace) a.unsat_trace[o] = utot + a.n_empty[f];
    }
  }
  for (int i = threadIdx.x; i < nf * RG; i += kPersistBlock) {
    const int rr = grp * RG + i % RG;
    if (rr < a.R) a.x[(int64_t)(vb + i / RG) * a.ldx + rr] = xa[i];
  }
}

}  // namespace

size_t persist_lds_bytes(int rg, int nf_max, int nocc_stage) {
  return persist_layout(rg, nf_max, nocc_stage).total;
}

hipError_t launch_persistent(const PersistArgs& a, int rg, hipStream_t s) {
  if (a.F <= 0 || a.steps <= 0) return hipSuccess;
  const int groups = (a.R + rg - 1) / rg;
  const size_t bytes = persist_lds_bytes(rg, a.nf_max, a.stage_occ ? a.nocc_max : 0);
  dim3 grid(a.F * groups), block(kPersistBlock);
#define GALSAT_PERSIST_CASE(N)                                                          \
  case N:                                                                               \
    if (a.stage_occ) hipLaunchKernelGGL((k_persistent<N, true>), grid, block, bytes, s, a); \
    else hipLaunchKernelGGL((k_persistent<N, false>), grid, block, bytes, s, a);            \
    break;
  switch (rg) {
    GALSAT_PERSIST_CASE(1)
    GALSAT_PERSIST_CASE(2)
    GALSAT_PERSIST_CASE(4)
    GALSAT_PERSIST_CASE(8)
    GALSAT_PERSIST_CASE(16)
    GALSAT_PERSIST_CASE(32)
    default: return hipErrorInvalidValue;
  }
#undef GALSAT_PERSIST_CASE
  return hipGetLastError();
}

}  // namespace galsat
