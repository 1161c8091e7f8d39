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

// The 16-bit storages with an even nx: one thread per pair of cells (x, x+1),
// x even, so each plane is read with one 4-byte load per thread (a whole
// 256-byte run per wavefront instruction).  Populations that stay in their
// column (c_x = 0) are stored as pairs; for the others each thread assembles
// the word of its own pair from one of its values and one of the adjacent
// lane's, so nearly every store is a full 4-byte word as well.  The
// arithmetic per cell is that of k3_bgk.
__device__ __forceinline__ constexpr int opp3(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// With PSM the pair also carries its solids (count, v_s in; F out, as in
// k3_psm) through 8-byte loads and stores, and collides as k3_psm does.
template <int P, bool PSM>
__device__ __forceinline__ void pairs_step(const typename Prec<P>::S *__restrict__ fin,
                                           typename Prec<P>::S *__restrict__ fout, int nx, int ny, int nz, float tau,
                                           const int32_t *__restrict__ n, const float *__restrict__ vs,
                                           float *__restrict__ force, float vol, float cap) {
  static_assert(sizeof(typename Prec<P>::S) == 2, "16-bit storage");
  using S = typename Prec<P>::S;
  const long long C = (long long)nx * ny * nz;
  const long long p = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (2 * p >= C) return;
  const long long c = 2 * p;  // even: x even, x + 1 in the same row
  const int x = (int)(c % nx);
  const long long yz = c / nx;
  const int y = (int)(yz % ny), z = (int)(yz / ny);
  const int q = x / 2, nq = nx / 2;       // pair index within the row
  const int lane = (int)(threadIdx.x & 63);
  float f0[Q3], f1[Q3];
#pragma unroll
  for (int i = 0; i < Q3; ++i) {
    struct alignas(4) S2 { S a, b; };
    const S2 v = *reinterpret_cast<const S2 *>(fin + (size_t)i * C + c);
    f0[i] = load_v<P>(&v.a, 0);
    f1[i] = load_v<P>(&v.b, 0);
  }
  const float omg = dv<P>(1.0f, tau);
  float gm[2] = {0.f, 0.f}, v[2][3] = {}, F[2][3] = {};
  if constexpr (PSM) {
    const int2 nn = *reinterpret_cast<const int2 *>(n + c);
    const int cnt[2] = {nn.x, nn.y};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      float es = (float)cnt[k] * vol;
      if (es > cap) es = cap;
      gm[k] = dv<P>(es * (tau - 0.5f), (1.f - es) + (tau - 0.5f));
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float2 t = *reinterpret_cast<const float2 *>(vs + (size_t)a * C + c);
      v[0][a] = t.x;
      v[1][a] = t.y;
    }
  }
  auto relax = [&](float *f, int k) {
    float r1 = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
    for (int i = 0; i < Q3; ++i) {
      r1 += f[i];
      jx += (float)c3(i, 0) * f[i];
      jy += (float)c3(i, 1) * f[i];
      jz += (float)c3(i, 2) * f[i];
    }
    const float rho = 1.f + r1;
    const float ir = dv<P>(1.0f, rho);
    const float ux = jx * ir, uy = jy * ir, uz = jz * ir;
    const float uu = ux * ux + uy * uy + uz * uz;
    if constexpr (PSM) {
      const float vx = v[k][0], vy = v[k][1], vz = v[k][2], gam = gm[k];
      const float vv = vx * vx + vy * vy + vz * vz;
      auto geq = [&](int i, float ax, float ay, float az, float aa) {
        const float cu = (float)c3(i, 0) * ax + (float)c3(i, 1) * ay + (float)c3(i, 2) * az;
        return w3<float>(i) * (r1 + rho * (3.f * cu + 4.5f * cu * cu - 1.5f * aa));
      };
      const float relax_ = dv<P>(1.f - gam, tau);
      float g[Q3], fx = 0.f, fy = 0.f, fz = 0.f;
#pragma unroll
      for (int i = 0; i < Q3; ++i) {
        const int o = opp3(i);
        const float om = f[o] - f[i] + geq(i, vx, vy, vz, vv) - geq(o, ux, uy, uz, uu);
        g[i] = f[i] - relax_ * (f[i] - geq(i, ux, uy, uz, uu)) + gam * om;
        fx += (float)c3(i, 0) * om;
        fy += (float)c3(i, 1) * om;
        fz += (float)c3(i, 2) * om;
      }
#pragma unroll
      for (int i = 0; i < Q3; ++i) f[i] = g[i];
      F[k][0] = gam * fx;
      F[k][1] = gam * fy;
      F[k][2] = gam * fz;
    } else {
#pragma unroll
      for (int i = 0; i < Q3; ++i) {
        const float cu = (float)c3(i, 0) * ux + (float)c3(i, 1) * uy + (float)c3(i, 2) * uz;
        const float geq = w3<float>(i) * (r1 + rho * (3.f * cu + 4.5f * cu * cu - 1.5f * uu));
        f[i] = f[i] - (f[i] - geq) * omg;
      }
    }
  };
  relax(f0, 0);
  relax(f1, 1);
  if constexpr (PSM) {
#pragma unroll
    for (int a = 0; a < 3; ++a) *reinterpret_cast<float2 *>(force + (size_t)a * C + c) = make_float2(F[0][a], F[1][a]);
  }
#pragma unroll
  for (int i = 0; i < Q3; ++i) {
    int ty = y + c3(i, 1), tz = z + c3(i, 2);
    ty = ty < 0 ? ty + ny : (ty >= ny ? ty - ny : ty);
    tz = tz < 0 ? tz + nz : (tz >= nz ? tz - nz : tz);
    const long long row = ((long long)tz * ny + ty) * nx;
    S *plane = fout + (size_t)i * C;
    if (c3(i, 0) == 0) {
      struct alignas(4) S2 { S a, b; };
      S2 v;
      store_v<P>(&v.a, 0, f0[i]);
      store_v<P>(&v.b, 0, f1[i]);
      *reinterpret_cast<S2 *>(plane + row + x) = v;
    } else {
      // The pair moves one cell along x, so its two values straddle two
      // aligned words. Each thread writes the word of its own pair, taking
      // the half that comes from the neighbouring pair from the adjacent
      // lane; at a wave's edge and at the row's periodic seam the value
      // without a partner in the wave goes out as a single 2-byte store.
      S t;
      store_v<P>(&t, 0, f0[i]);
      const unsigned s0 = *reinterpret_cast<const unsigned short *>(&t);
      store_v<P>(&t, 0, f1[i]);
      const unsigned s1 = *reinterpret_cast<const unsigned short *>(&t);
      unsigned *word = reinterpret_cast<unsigned *>(plane + row + x);
      if (c3(i, 0) > 0) {
        // cell x-1 (previous pair's second) -> x, cell x -> x+1, cell x+1 -> x+2
        const unsigned prev = (unsigned)__shfl_up((int)s1, 1, 64);
        if (lane > 0 && q > 0) {
          *word = (prev & 0xffffu) | (s0 << 16);
        } else {
          store_v<P>(plane, (size_t)(row + x + 1), f0[i]);
        }
        if (lane == 63 || q == nq - 1) store_v<P>(plane, (size_t)(row + (x + 2 == nx ? 0 : x + 2)), f1[i]);
      } else {
        // cell x+1 -> x, cell x+2 (next pair's first) -> x+1, cell x -> x-1
        const unsigned next = (unsigned)__shfl_down((int)s0, 1, 64);
        if (lane < 63 && q < nq - 1) {
          *word = s1 | ((next & 0xffffu) << 16);
        } else {
          store_v<P>(plane, (size_t)(row + x), f1[i]);
        }
        if (lane == 0 || q == 0) store_v<P>(plane, (size_t)(row + (x == 0 ? nx - 1 : x - 1)), f0[i]);
      }
    }
  }
}

template <int P>
__global__ __launch_bounds__(BLOCK) void k3_bgk_pairs(const typename Prec<P>::S *__restrict__ fin,
                                                      typename Prec<P>::S *__restrict__ fout, int nx, int ny, int nz,
                                                      float tau) {
  pairs_step<P, false>(fin, fout, nx, ny, nz, tau, nullptr, nullptr, nullptr, 0.f, 0.f);
}

template <int P>
__global__ __launch_bounds__(BLOCK) void k3_psm_pairs(const typename Prec<P>::S *__restrict__ fin,
                                                      typename Prec<P>::S *__restrict__ fout, int nx, int ny, int nz,
                                                      float tau, const int32_t *__restrict__ n,
                                                      const float *__restrict__ vs, float *__restrict__ force,
                                                      float vol, float cap) {
  pairs_step<P, true>(fin, fout, nx, ny, nz, tau, n, vs, force, vol, cap);
}

// One partially saturated step of the 3-D lattice (the collision of Eqs. 6-7
// with the weighting of Eq. 9 and the force of Eq. 25, on D3Q19): cell c
// holds n[c] spheres of volume vol moving with vs[.][c]; its solid fraction
// is n vol, at most cap; the momentum the solids give the gas goes to
// force[.][c].  FP64 follows the oracle's operation order (bit for bit); the
// reduced storages work on deviations, where Eq. 7's term reads
// g_opp - g_i + g^eq_i(v_s) - g^eq_opp(u) because w_i = w_opp.
template <int P>
__global__ __launch_bounds__(BLOCK) void k3_psm(const typename Prec<P>::S *__restrict__ fin,
                                                typename Prec<P>::S *__restrict__ fout,
                                                const int32_t *__restrict__ n,
                                                const typename Prec<P>::T *__restrict__ vs,
                                                typename Prec<P>::T *__restrict__ force, int nx, int ny, int nz,
                                                typename Prec<P>::T tau, typename Prec<P>::T vol,
                                                typename Prec<P>::T cap) {
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
  T es = (T)n[c] * vol;
  if (es > cap) es = cap;
  const T half = (T)0.5;
  const T gam = dv<P>(es * (tau - half), ((T)1 - es) + (tau - half));
  const T vx = vs[c], vy = vs[C + c], vz = vs[2 * C + c];
  T out[Q3];
  T fx = (T)0, fy = (T)0, fz = (T)0;
  if constexpr (P == PREC_FP64) {
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
    const T vv = vx * vx + vy * vy + vz * vz;
    auto feq = [&](int i, T ax, T ay, T az, T aa) {
      const T cu = (T)c3(i, 0) * ax + (T)c3(i, 1) * ay + (T)c3(i, 2) * az;
      return w3<T>(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * aa);
    };
    const T relax = (1.0 - gam) / tau;
#pragma unroll
    for (int i = 0; i < Q3; ++i) {
      const int o = opp3(i);
      const T om = f[o] - f[i] + feq(i, vx, vy, vz, vv) - feq(o, ux, uy, uz, uu);
      out[i] = f[i] - relax * (f[i] - feq(i, ux, uy, uz, uu)) + gam * om;
      fx += (T)c3(i, 0) * om;
      fy += (T)c3(i, 1) * om;
      fz += (T)c3(i, 2) * om;
    }
  } else {
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
    const T vv = vx * vx + vy * vy + vz * vz;
    auto geq = [&](int i, T ax, T ay, T az, T aa) {
      const T cu = (T)c3(i, 0) * ax + (T)c3(i, 1) * ay + (T)c3(i, 2) * az;
      return w3<T>(i) * (r1 + rho * ((T)3 * cu + (T)4.5 * cu * cu - (T)1.5 * aa));
    };
    const T relax = dv<P>((T)1 - gam, tau);
#pragma unroll
    for (int i = 0; i < Q3; ++i) {
      const int o = opp3(i);
      const T om = f[o] - f[i] + geq(i, vx, vy, vz, vv) - geq(o, ux, uy, uz, uu);
      out[i] = f[i] - relax * (f[i] - geq(i, ux, uy, uz, uu)) + gam * om;
      fx += (T)c3(i, 0) * om;
      fy += (T)c3(i, 1) * om;
      fz += (T)c3(i, 2) * om;
    }
  }
  force[c] = gam * fx;
  force[C + c] = gam * fy;
  force[2 * C + c] = gam * fz;
#pragma unroll
  for (int i = 0; i < Q3; ++i) {
    int tx = x + c3(i, 0), ty = y + c3(i, 1), tz = z + c3(i, 2);
    tx = tx < 0 ? tx + nx : (tx >= nx ? tx - nx : tx);
    ty = ty < 0 ? ty + ny : (ty >= ny ? ty - ny : ty);
    tz = tz < 0 ? tz + nz : (tz >= nz ? tz - nz : tz);
    store_v<P>(fout, (size_t)i * C + ((long long)tz * ny + ty) * nx + tx, out[i]);
  }
}


}  // namespace lbdps
