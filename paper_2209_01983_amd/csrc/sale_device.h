// sale_device.h -- device helpers shared by the libsale kernels: index math,
// the closed-form swept volume, wave64 reductions, XCD-aware block order.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "../../include/sale.h"
#include "sale_impl.h"

namespace sale {

__device__ __forceinline__ int64_t cidx(const Mesh &m, int i, int j, int k) {
  return i + (int64_t)m.nx * (j + (int64_t)m.ny * k);
}
__device__ __forceinline__ int64_t nidx(const Mesh &m, int i, int j, int k) {
  return i + (int64_t)(m.nx + 1) * (j + (int64_t)(m.ny + 1) * k);
}
__device__ __forceinline__ bool cell_in(const Mesh &m, int i, int j, int k) {
  return i >= 0 && i < m.nx && j >= 0 && j < m.ny && k >= 0 && k < m.nz;
}

// Exact volume swept by a rectangular face (edge lengths h1 along its first
// tangent s, h2 along its second t; tangents cyclic after the normal) whose
// corners (s,t) = (0,0), (1,0), (0,1), (1,1) move by d0..d3 (components:
// normal, t1, t2). With delta(s,t) = A + B s + C t + E s t the swept volume is
//   h1 h2 <xi> + h1/2 <xi zeta_t - zeta xi_t> + h2/2 <xi eta_s - eta xi_s>
//   + 1/3 <delta . (delta_s x delta_t)>,   <.> = integral over [0,1]^2.
// The two middle brackets reduce to 1D integrals along the edges t = 0 and
// s = 0 (their s t terms cancel) and the triple product integrates to
// A.(B x C) + 1/2 A.((B - C) x E) + 1/4 C.(B x E).
// h12 = h1 h2, hh1 = h1 / 2, hh2 = h2 / 2.
template <typename R>
__device__ __forceinline__ R swept_volume(const R d0[3], const R d1[3], const R d2[3], const R d3[3],
                                          R h12, R hh1, R hh2) {
  R A[3], B[3], C[3], E[3];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    A[a] = d0[a];
    B[a] = d1[a] - d0[a];
    C[a] = d2[a] - d0[a];
    E[a] = (d3[a] - d1[a]) - C[a];
  }
  const R half = R(0.5), third = R(1) / R(3), quarter = R(0.25);
  const R t0 = h12 * (quarter * ((d0[0] + d1[0]) + (d2[0] + d3[0])));
  const R i1 = (A[0] * C[2] + half * (A[0] * E[2] + B[0] * C[2]) + third * B[0] * E[2]) -
               (A[2] * C[0] + half * (A[2] * E[0] + B[2] * C[0]) + third * B[2] * E[0]);
  const R i2 = (A[0] * B[1] + half * (A[0] * E[1] + C[0] * B[1]) + third * C[0] * E[1]) -
               (A[1] * B[0] + half * (A[1] * E[0] + C[1] * B[0]) + third * C[1] * E[0]);
  const R BC0 = B[1] * C[2] - B[2] * C[1], BC1 = B[2] * C[0] - B[0] * C[2], BC2 = B[0] * C[1] - B[1] * C[0];
  const R D0 = B[0] - C[0], D1 = B[1] - C[1], D2 = B[2] - C[2];
  const R DE0 = D1 * E[2] - D2 * E[1], DE1 = D2 * E[0] - D0 * E[2], DE2 = D0 * E[1] - D1 * E[0];
  const R BE0 = B[1] * E[2] - B[2] * E[1], BE1 = B[2] * E[0] - B[0] * E[2], BE2 = B[0] * E[1] - B[1] * E[0];
  const R trip = (A[0] * BC0 + A[1] * BC1 + A[2] * BC2) + half * (A[0] * DE0 + A[1] * DE1 + A[2] * DE2) +
                 quarter * (C[0] * BE0 + C[1] * BE1 + C[2] * BE2);
  return t0 + hh1 * i1 + hh2 * i2 + third * trip;
}

// a * b rounded on its own: the empty statement hides the product from the
// compiler, which would otherwise fuse it with a following add (the build
// contracts across statements, and a per-function pragma does not stop the
// code generator from doing so)
__device__ __forceinline__ double mul_rn(double a, double b) {
  double p = a * b;
  asm volatile("" : "+v"(p));
  return p;
}

// Cell divergence D = (1/V0) sum_p S_cp . u_p from the halves of its corner
// sums on the cell's lower (a) and upper (b) node planes: x and y halves are
// pairwise edge differences, z halves the sums of w over the plane's four
// nodes. Written with explicit FMAs so that every kernel forming D of the
// same state gets the same bits (a restart must reproduce a run exactly).
template <typename R>
__device__ __forceinline__ R divergence(const Mesh &m, R xa, R xb, R ya, R yb, R za, R zb) {
  return fma(R(m.az), zb - za, fma(R(m.ay), ya + yb, R(m.ax) * (xa + xb))) * R(m.iV0);
}

// divergence D of cell (i,j,k) of state s, formed as in the step kernels
template <typename R>
__device__ __forceinline__ R state_divergence(const Mesh &m, const State<R> &s, int i, int j, int k) {
  R x[2], y[2], z[2];
#pragma unroll
  for (int c = 0; c < 2; c++) {
    auto at = [&](const R *f, int a, int b) { return f[nidx(m, i + a, j + b, k + c)]; };
    x[c] = (at(s.u, 1, 0) - at(s.u, 0, 0)) + (at(s.u, 1, 1) - at(s.u, 0, 1));
    y[c] = (at(s.v, 0, 1) - at(s.v, 0, 0)) + (at(s.v, 1, 1) - at(s.v, 1, 0));
    z[c] = ((at(s.w, 0, 0) + at(s.w, 1, 0)) + at(s.w, 0, 1)) + at(s.w, 1, 1);
  }
  return divergence(m, x[0], x[1], y[0], y[1], z[0], z[1]);
}

// node speed |u|, same bits in every kernel
template <typename R>
__device__ __forceinline__ R speed(R u, R v, R w) {
  return sqrt(fma(w, w, fma(v, v, u * u)));
}

template <typename R>
__device__ __forceinline__ R wave_max(R x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}
template <typename R>
__device__ __forceinline__ R wave_sum(R x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Block-wide max of a >= 0 folded into ctl->amax_bits (the bit patterns of
// non-negative doubles order like their values), and a NUMERIC flag if any
// thread saw an inadmissible cell. NT = threads per block (multiple of 64).
template <int NT>
__device__ __forceinline__ void block_max_to_ctl(Ctl *ctl, double a, bool bad) {
  __shared__ double red[NT / 64];
  __shared__ int anybad;
  if (threadIdx.x == 0) anybad = 0;
  __syncthreads();
  if (bad) anybad = 1;
  a = wave_max(bad ? 0.0 : a);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int q = 1; q < NT / 64; q++) r = fmax(r, red[q]);
    if (r > 0.0) atomicMax(&ctl->amax_bits, (unsigned long long)__double_as_longlong(r));
    if (anybad) atomicOr(&ctl->status, SALE_FLAG_NUMERIC);
  }
}

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8), each with its own L2. Renumber so that consecutive logical tiles --
// which share halo planes -- land on the same XCD.
__device__ __forceinline__ int xcd_logical_block(int b, int nblocks) {
  const int per = (nblocks + 7) / 8;
  const int xcd = b % 8, slot = b / 8;
  const int full = nblocks - 8 * (per - 1);  // XCDs that received `per` blocks
  return (xcd < full ? xcd * per : full * per + (xcd - full) * (per - 1)) + slot;
}

}  // namespace sale
