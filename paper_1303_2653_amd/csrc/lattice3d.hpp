// The 3-D gas lattice (D3Q19), the first piece of the 3-D extension: one BGK
// collide-stream step on a periodic box.  The same storage patterns as the
// 2-D path: FP64 values, or deviations g_i = f_i - w_i in FP32, FP16 or BF16
// with FP32 arithmetic.  One thread per cell of an x-row run: it reads its 19
// populations (each plane contiguous in x), relaxes towards f^eq with 1/tau
// and pushes f*_i to the cell x + c_i, so every load and store of a plane is a
// contiguous run per wavefront.
#pragma once

#include "device.hpp"

namespace lbdps {

constexpr int Q3 = 19;
__host__ __device__ constexpr int c3(int i, int a) {
  // rest, 6 faces, 12 edges (the order of the oracle's table)
  constexpr signed char t[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0},  {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
                                    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},  {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
                                    {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
  return t[i][a];
}
template <class T> __host__ __device__ constexpr T w3(int i) {
  return i == 0 ? (T)1 / (T)3 : (i < 7 ? (T)1 / (T)18 : (T)1 / (T)36);
}

template <int P>
__global__ __launch_bounds__(BLOCK) void k3_bgk(const typename Prec<P>::S *__restrict__ fin,
                                                typename Prec<P>::S *__restrict__ fout, int nx, int ny, int nz,
                                                typename Prec<P>::T tau) {
  using T = typename Prec<P>::T;
  const long long C = (long long)nx * ny * nz;
  const long long c = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (c >= C) return;
  const int x = (int)(c % nx);
  const long long yz = c / nx;
  const int y = (int)(yz % ny), z = (int)(yz / ny);
  T f[Q3];
#pragma unroll
  for (int i = 0; i < Q3; ++i) f[i] = load_v<P>(fin, (size_t)i * C + c);
  T out[Q3];
  if constexpr (P == PREC_FP64) {
    // the oracle's operations in its order (FP64 results bit for bit)
    T rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < Q3; ++i) {
      rho += f[i];
      jx += (T)c3(i, 0) * f[i];
      jy += (T)c3(i, 1) * f[i];
      jz += (T)c3(i, 2) * f[i];
    }
    const T ux = jx / rho, uy = jy / rho, uz = jz / rho;
    const T uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int i = 0; i < Q3; ++i) {
      const T cu = (T)c3(i, 0) * ux + (T)c3(i, 1) * uy + (T)c3(i, 2) * uz;
      const T feq = w3<T>(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
      out[i] = f[i] - (f[i] - feq) / tau;
    }
  } else {
    // deviations: rho - 1 = sum g, j = sum c g; g^eq = w ((rho - 1) + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u))
    T r1 = (T)0, jx = (T)0, jy = (T)0, jz = (T)0;
#pragma unroll
    for (int i = 0; i < Q3; ++i) {
      r1 += f[i];
      jx += (T)c3(i, 0) * f[i];
      jy += (T)c3(i, 1) * f[i];
      jz += (T)c3(i, 2) * f[i];
    }
    const T rho = (T)1 + r1;
    const T ir = dv<P>((T)1, rho);
    const T ux = jx * ir, uy = jy * ir, uz = jz * ir;
    const T uu = ux * ux + uy * uy + uz * uz;
    const T omg = dv<P>((T)1, tau);
#pragma unroll
    for (int i = 0; i < Q3; ++i) {
      const T cu = (T)c3(i, 0) * ux + (T)c3(i, 1) * uy + (T)c3(i, 2) * uz;
      const T geq = w3<T>(i) * (r1 + rho * ((T)3 * cu + (T)4.5 * cu * cu - (T)1.5 * uu));
      out[i] = f[i] - (f[i] - geq) * omg;
    }
  }
  // push to x + c_i, periodic in every axis
  const bool inner = x >= 1 && x < nx - 1 && y >= 1 && y < ny - 1 && z >= 1 && z < nz - 1;
#pragma unroll
  for (int i = 0; i < Q3; ++i) {
    long long d;
    if (inner) {
      d = c + c3(i, 0) + (long long)c3(i, 1) * nx + (long long)c3(i, 2) * nx * ny;
    } else {
      int tx = x + c3(i, 0), ty = y + c3(i, 1), tz = z + c3(i, 2);
      tx = tx < 0 ? tx + nx : (tx >= nx ? tx - nx : tx);
      ty = ty < 0 ? ty + ny : (ty >= ny ? ty - ny : ty);
      tz = tz < 0 ? tz + nz : (tz >= nz ? tz - nz : tz);
      d = ((long long)tz * ny + ty) * nx + tx;
    }
    store_v<P>(fout, (size_t)i * C + d, out[i]);
  }
}

}  // namespace lbdps
