// Vector kernels of the serving loop's conjugate-gradient solves.
//
// Every active CG request owns FP64 vectors b, x, r, p, d, q64 and FP32
// p32, q32 of its own length.  A step processes all requests at once: the
// vectors are cut into tiles of kTile elements, a per-tile request table maps
// workgroups to (request, tile), and every reduction is done per tile in a
// fixed order, then per request over its tiles in a fixed order.  The
// per-request sums (p.q for alpha, r.r for beta) are formed by every workgroup
// of the request that needs them, each in the same order, so a step needs no
// kernel of its own for the scalars; the ones the host needs (|r|^2, |b|^2,
// p.q) are also written straight into a mapped pinned mirror, so a step needs
// no copy back either.  A step may run several inner iterations (passes) of
// a request back to back: the direction kernel of pass j records whether the
// request's inner cycle stops there (p.q <= 0 or |r|^2 at or below the
// cycle's threshold, the same tests the host applies), and the kernels of
// pass j+1 skip a request that stopped, so the iterations and their
// arithmetic are exactly those of one pass per step.  No value of one request ever enters
// another request's arithmetic, so each result is bitwise the same whether
// the request runs alone or in a mix.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace argcsr {

constexpr int kVecBlock = 256;
constexpr int kVecPerThread = 8;
constexpr int kTile = kVecBlock * kVecPerThread;
constexpr int kMaxInnerPerStep = 8;   // inner CG passes one step may run

enum CgPhase : int32_t {
  kPhaseStart = 0,   // r = b, p = r, d = 0, rr = |b|^2 = bnorm2
  kPhaseInner = 1,   // one CG iteration on the FP32 matrix
  kPhaseOuter = 2,   // x += d, r = b - A64 x (FP64 matrix), restart: p = r, d = 0
};

struct CgVec {
  const double* b;
  double* x;
  double* r;
  double* p;
  double* d;
  const double* q64;     // A64 x (outer phase)
  float* p32;            // FP32 copy of p, the FP32 SpMV's input
  const float* q32;      // A32 p32 (inner phase)
  int32_t n;
  int32_t phase;
  int32_t tile_begin;    // first global tile of this request
  int32_t slot;          // index into the scalar array
  int32_t parity;        // rr[parity] is |r|^2 before this pass; the pass writes rr[1 - parity]
  int32_t pass;          // 1-based inner pass of the step (1 for the other phases)
  double stop_rr;        // inner: the cycle stops once |r|^2 <= stop_rr
};

struct CgScalars {
  double rr[2];          // recursive (inner) or true (outer) |r|^2, by pass parity
  double alpha;
  double beta;
  double bnorm2;         // |b|^2
  double pq;             // p . A32 p of the last inner iteration
  int32_t passes;        // inner passes the last step ran for this request
  int32_t stop[kMaxInnerPerStep + 1];   // stop[j]: the cycle ended at or before pass j
  int32_t pad[2];
};

// Passes after the first skip a request whose cycle has ended.
__device__ __forceinline__ bool cg_skip(const CgVec& w, const CgScalars* sc) {
  return w.pass > 1 && sc[w.slot].stop[w.pass - 1] != 0;
}

// Fixed-order block sum: each thread's values in index order, then a
// tree over the 256 threads.
__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = kVecBlock / 2; s > 0; s >>= 1) {
    if (int(threadIdx.x) < s) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + s];
    __syncthreads();
  }
  return red[0];
}

// x += d for requests entering the outer phase (before the FP64 SpMV reads x).
static __global__ __launch_bounds__(kVecBlock) void cg_pre_kernel(const CgVec* __restrict__ v,
                                                          const int32_t* __restrict__ tile_req) {
  const CgVec w = v[tile_req[blockIdx.x]];
  if (w.phase != kPhaseOuter) return;
  const int32_t base = (int32_t(blockIdx.x) - w.tile_begin) * kTile;
  for (int k = 0; k < kVecPerThread; ++k) {
    const int32_t i = base + k * kVecBlock + int32_t(threadIdx.x);
    if (i < w.n) w.x[i] = w.x[i] + w.d[i];
  }
}

// inner: partial sums of p . q32 into `partial`
static __global__ __launch_bounds__(kVecBlock) void cg_dot_kernel(const CgVec* __restrict__ v,
                                                          const int32_t* __restrict__ tile_req,
                                                          const CgScalars* __restrict__ sc,
                                                          double* __restrict__ partial) {
  __shared__ double red[kVecBlock];
  const CgVec w = v[tile_req[blockIdx.x]];
  if (w.phase != kPhaseInner || cg_skip(w, sc)) return;
  const int32_t base = (int32_t(blockIdx.x) - w.tile_begin) * kTile;
  double s = 0.0;
  for (int k = 0; k < kVecPerThread; ++k) {
    const int32_t i = base + k * kVecBlock + int32_t(threadIdx.x);
    if (i < w.n) s = __builtin_fma(w.p[i], double(w.q32[i]), s);
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Sum of one request's tile partials, by one workgroup: thread t adds tiles
// t, t+256, ... in order, then a fixed tree over the threads.  The order
// depends only on the request's own tile count, so every workgroup of the
// request gets the same value.  Ends with a barrier, so `red` may be reused.
__device__ __forceinline__ double tiles_sum(const double* partial, int32_t begin, int32_t n,
                                           double* red) {
  const int32_t tiles = (n + kTile - 1) / kTile;
  double s = 0.0;
  for (int32_t t = int32_t(threadIdx.x); t < tiles; t += kVecBlock) s += partial[begin + t];
  s = block_sum(s, red);
  __syncthreads();
  return s;
}

// inner: alpha = rr / (p . q) from the request's p.q partials, then
// d += alpha p, r -= alpha q32; start/outer: r = b (- q64), d = 0, p = r,
// p32 = (float) r.  All phases: partial sums of r . r into `rr_partial`.
static __global__ __launch_bounds__(kVecBlock) void cg_update_kernel(const CgVec* __restrict__ v,
                                                             const int32_t* __restrict__ tile_req,
                                                             CgScalars* __restrict__ sc,
                                                             CgScalars* __restrict__ host_sc,
                                                             const double* __restrict__ pq_partial,
                                                             double* __restrict__ rr_partial) {
  __shared__ double red[kVecBlock];
  const CgVec w = v[tile_req[blockIdx.x]];
  if (cg_skip(w, sc)) return;                       // uniform: one request per workgroup
  const int32_t local = int32_t(blockIdx.x) - w.tile_begin;
  const int32_t base = local * kTile;
  double s = 0.0;
  if (w.phase == kPhaseInner) {
    const double pq = tiles_sum(pq_partial, w.tile_begin, w.n, red);
    const double alpha = pq > 0.0 ? sc[w.slot].rr[w.parity] / pq : 0.0;   // pq <= 0: no step
    if (local == 0 && threadIdx.x == 0) {                                  // (host leaves the cycle)
      sc[w.slot].pq = pq;
      sc[w.slot].alpha = alpha;
      host_sc[w.slot].pq = pq;
    }
    for (int k = 0; k < kVecPerThread; ++k) {
      const int32_t i = base + k * kVecBlock + int32_t(threadIdx.x);
      if (i < w.n) {
        w.d[i] = __builtin_fma(alpha, w.p[i], w.d[i]);
        const double ri = __builtin_fma(-alpha, double(w.q32[i]), w.r[i]);
        w.r[i] = ri;
        s = __builtin_fma(ri, ri, s);
      }
    }
  } else {
    const bool outer = w.phase == kPhaseOuter;
    for (int k = 0; k < kVecPerThread; ++k) {
      const int32_t i = base + k * kVecBlock + int32_t(threadIdx.x);
      if (i < w.n) {
        const double ri = outer ? w.b[i] - w.q64[i] : w.b[i];
        w.r[i] = ri;
        w.p[i] = ri;
        w.p32[i] = float(ri);
        w.d[i] = 0.0;
        s = __builtin_fma(ri, ri, s);
      }
    }
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) rr_partial[blockIdx.x] = s;
}

// All phases: rr_new = r . r from the request's partials, stored as
// rr[1 - parity] (and as |b|^2 at the start); inner: whether the cycle stops
// at this pass (stop[pass]), beta = rr_new / rr, p = r + beta p,
// p32 = (float) p.  A skipped pass passes the stop on to the next one.
static __global__ __launch_bounds__(kVecBlock) void cg_direction_kernel(const CgVec* __restrict__ v,
                                                                const int32_t* __restrict__ tile_req,
                                                                CgScalars* __restrict__ sc,
                                                                CgScalars* __restrict__ host_sc,
                                                                const double* __restrict__ rr_partial) {
  __shared__ double red[kVecBlock];
  const CgVec w = v[tile_req[blockIdx.x]];
  const int32_t local = int32_t(blockIdx.x) - w.tile_begin;
  if (cg_skip(w, sc)) {        // this pass's kernels read stop[pass - 1] only, never stop[pass]
    if (local == 0 && threadIdx.x == 0) sc[w.slot].stop[w.pass] = 1;
    return;
  }
  const double rr_new = tiles_sum(rr_partial, w.tile_begin, w.n, red);
  if (local == 0 && threadIdx.x == 0) {
    sc[w.slot].rr[1 - w.parity] = rr_new;
    host_sc[w.slot].rr[1 - w.parity] = rr_new;
    if (w.phase == kPhaseStart) {
      sc[w.slot].bnorm2 = rr_new;
      host_sc[w.slot].bnorm2 = rr_new;
    }
    if (w.phase == kPhaseInner) {
      sc[w.slot].stop[w.pass] = (sc[w.slot].pq <= 0.0 || rr_new <= w.stop_rr) ? 1 : 0;
      host_sc[w.slot].passes = w.pass;
    }
  }
  if (w.phase != kPhaseInner) return;
  const double rr = sc[w.slot].rr[w.parity];
  const double beta = rr > 0.0 ? rr_new / rr : 0.0;
  if (local == 0 && threadIdx.x == 0) sc[w.slot].beta = beta;
  const int32_t base = local * kTile;
  for (int k = 0; k < kVecPerThread; ++k) {
    const int32_t i = base + k * kVecBlock + int32_t(threadIdx.x);
    if (i < w.n) {
      const double pi = __builtin_fma(beta, w.p[i], w.r[i]);
      w.p[i] = pi;
      w.p32[i] = float(pi);
    }
  }
}

// The step's descriptor block, read by the device from mapped pinned host
// memory: one small kernel costs the host less than a copy call.
static __global__ __launch_bounds__(kVecBlock) void desc_pull_kernel(const int4* __restrict__ src,
                                                             int4* __restrict__ dst, int64_t n16) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n16;
       i += int64_t(gridDim.x) * blockDim.x)
    dst[i] = src[i];
}

// FP64 values -> FP32 values of the same layout (nearest-even).
static __global__ __launch_bounds__(kVecBlock) void round_values_kernel(const double* __restrict__ v64,
                                                                float* __restrict__ v32,
                                                                int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    v32[i] = float(v64[i]);
}

}  // namespace argcsr
