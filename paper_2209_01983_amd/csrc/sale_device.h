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
// normal xi, t1 eta, t2 zeta). The swept volume is
//   h1 h2 <xi> + h1/2 <xi zeta_t - zeta xi_t> + h2/2 <xi eta_s - eta xi_s>
//   + 1/3 <delta . (delta_s x delta_t)>,   <.> = integral over [0,1]^2,
// and for the bilinear delta each bracket has a closed form in the corners:
//   <xi>                        = (d0 + d1 + d2 + d3)_xi / 4
//   <xi zeta_t - zeta xi_t>     = [m0 x m1]_(xi,zeta) / 4 + [b x e]_(xi,zeta) / 12
//   <xi eta_s - eta xi_s>       = [n0 x n1]_(xi,eta) / 4 + [c x e]_(xi,eta) / 12
//   <delta . (delta_s x delta_t)> = (d0 + d1 + d2 + d3) . ((d3 - d0) x (d2 - d1)) / 8
// with the edge sums m0 = d0 + d1, m1 = d2 + d3 (edges along s), n0 = d0 + d2,
// n1 = d1 + d3 (edges along t), the edge differences b = d1 - d0, c = d2 - d0,
// the twist e = d3 - d2 - d1 + d0, and [p x q]_(a,b) = p_a q_b - p_b q_a. (The
// last line is the cone volume of a bilinear patch through its diagonals.)
// q12 = h1 h2 / 4, e1 = h1 / 8, e2 = h2 / 8.
template <typename R>
__device__ __forceinline__ R swept_volume(const R d0[3], const R d1[3], const R d2[3], const R d3[3],
                                          R q12, R e1, R e2) {
  const R third = R(1) / R(3);
  // (xi, zeta) brackets
  const R m0x = d0[0] + d1[0], m1x = d2[0] + d3[0], m0z = d0[2] + d1[2], m1z = d2[2] + d3[2];
  const R bx = d1[0] - d0[0], bz = d1[2] - d0[2];
  const R ex = (d3[0] - d2[0]) - bx, ez = (d3[2] - d2[2]) - bz;
  const R Sx = m0x + m1x, Sz = m0z + m1z;
  R v = q12 * Sx + e1 * ((m0x * m1z - m0z * m1x) + third * (bx * ez - bz * ex));
  // (xi, eta) brackets
  const R n0x = d0[0] + d2[0], n1x = d1[0] + d3[0], n0y = d0[1] + d2[1], n1y = d1[1] + d3[1];
  const R ey = (d3[1] - d2[1]) - (d1[1] - d0[1]);
  const R Sy = n0y + n1y;
  v += e2 * ((n0x * n1y - n0y * n1x) + third * ((d2[0] - d0[0]) * ey - (d2[1] - d0[1]) * ex));
  // cone volume through the diagonals
  const R gx = d3[0] - d0[0], gy = d3[1] - d0[1], gz = d3[2] - d0[2];
  const R fx = d2[0] - d1[0], fy = d2[1] - d1[1], fz = d2[2] - d1[2];
  const R trip = (Sx * (gy * fz - gz * fy) + Sy * (gz * fx - gx * fz)) + Sz * (gx * fy - gy * fx);
  return v + third * (R(0.125) * trip);
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
