// The 3-D coupled step: the procedure of Sec. 2.4 on a fully periodic D3Q19
// box with spheres (the fully 3-D simulation the paper names as the natural
// extension, Sec. 4).  The same layout ideas as the 2-D path: populations in
// planes [19][nz][ny][nx] (FP64, or deviations f_i - w_i in FP32, FP16 or
// BF16 with FP32 arithmetic), node fields in planes, particle records in
// structure-of-arrays form kept sorted by cell, so that deposition is a
// segment read and the drag correction of Eq. 28 a per-cell pass.  Positions
// are global coordinates in FP64 and cell + offset in the FP32 modes.  The
// FP64 arithmetic follows the oracle's order, so FP64 results equal its bit
// for bit (or to a few ulp where pow and sqrt enter).
//
// One step is seven launches:
//   k3c_collide   deposition (segment sorted by particle index, n, v_s), the
//                 collision of Eq. 23 with the solid term of Eq. 7, F_pg
//                 (Eq. 25), u_sup (Eq. 24), u_gas, beta (Eqs. 19, 21, 22),
//                 push streaming on the periodic box;
//   k3c_gradp     grad p of p = rho / 3, central differences;
//   k3c_drag      trilinear interpolation, Eqs. 26-28, Eq. 16, the move, the
//                 count of each particle's new cell;
//   scan, k3c_scatter   the records to their new cell order;
//   k3c_contacts  the contact rows (the cells within d of a particle);
//   k3c_clusters  binary collisions (Eqs. 17-18) of each small contact cluster
//                 in lexicographic pair order;
//   k3c_resolve   the ordered sweep for clusters too large for k3c_clusters.
#pragma once

#include "kernels.hpp"
#include "lattice3d.hpp"

namespace lbdps {

// Per-count table of the 3-D step (FP64 on the host, in the arithmetic type):
// the solid volume fraction, the BGK factor (1 - gamma) / tau, omega gamma,
// the voidage, and the drag-law constants of Eqs. 19, 21, 22 at that count.
enum { L3_ES = 0, L3_RELAX, L3_OMG, L3_EG, L3_DILUTE, L3_A, L3_BRE, L3_H, L3_OM, L3_D1, L3_D2, L3_W };

// XCD run lengths of the 3-D kernels that read neighbouring rows and planes.
// The gradient reads the rows above and below, which runs of 8 tiles keep on
// one XCD; the contact search (27 cells) takes one contiguous run of tiles per
// XCD.  On the 256 x 256 x 1024 riser each is 3-4 % faster than in dispatch
// order; the drag, whose node reads are spread over whole planes, gains
// nothing from either and keeps the dispatch order.
constexpr int XCD_RUN_3D_CONTACTS = 0, XCD_RUN_3D_GRADP = 8;

template <class T> struct Parts3 {
  int32_t *key, *pid;  // cell (z ny + y) nx + x; particle index
  T *px, *py, *pz;     // global position (FP64) or offset in the cell
  T *vx, *vy, *vz;
};

// node: per cell the eight values the particle interpolation reads, packed
// (u_gas x, y, z, solid fraction, beta, grad p x, y, z) so that a node is one
// contiguous 8-value load.
template <class T> struct Fields3 {
  T *rho, *ugx, *ugy, *ugz, *beta, *es, *fpx, *fpy, *fpz, *node;
};
template <class T> struct alignas(8 * sizeof(T)) Node8 {
  T v[8];
};

template <class T> struct Consts3 {
  int nx, ny, nz, C, npart, nlut;
  T tau, d, dd, mu, vp, m, msum, one_e, fp;
  T geff[3], halfG[3], src[Q3];
  int32_t *flags;
  unsigned spin_limit;
};

template <class T> __device__ __forceinline__ void cell3_xyz(const Consts3<T> &k, int key, int &x, int &y, int &z) {
  x = key % k.nx;
  const int yz = key / k.nx;
  y = yz % k.ny;
  z = yz / k.ny;
}
__device__ __forceinline__ int wrap_p(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

template <int P> struct Pos3 {
  using T = typename Prec<P>::T;
  static constexpr bool G = Prec<P>::global_pos;

  // Minimum-image separation a - b on every axis.
  __device__ static void sep(const Consts3<T> &k, int ka, const T *a, int kb, const T *b, T *d) {
    const int n[3] = {k.nx, k.ny, k.nz};
    if constexpr (G) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        T x = a[q] - b[q];
        if (x > (T)0.5 * (T)n[q])
          x -= (T)n[q];
        else if (x < -(T)0.5 * (T)n[q])
          x += (T)n[q];
        d[q] = x;
      }
    } else {
      int ca[3], cb[3];
      cell3_xyz(k, ka, ca[0], ca[1], ca[2]);
      cell3_xyz(k, kb, cb[0], cb[1], cb[2]);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        int dc = ca[q] - cb[q];
        if (dc > n[q] / 2)
          dc -= n[q];
        else if (dc < -(n[q] / 2))
          dc += n[q];
        d[q] = (T)dc + (a[q] - b[q]);
      }
    }
  }

  // Trilinear stencil origin and fractions for s = P - 1/2 along one axis;
  // c is the particle's cell on that axis.
  __device__ static void axis_stencil(int c, T o, int &i0, T &t) {
    if constexpr (G) {
      const T s = o - (T)0.5, fl = floor(s);
      t = s - fl;
      i0 = (int)fl;
    } else if (o >= (T)0.5) {
      i0 = c;
      t = o - (T)0.5;
    } else {
      i0 = c - 1;
      t = o + (T)0.5;
    }
  }

  // P <- P + v on one periodic axis; returns the new cell on that axis, or -1
  // if the result is not a position in the box (NaN, or a jump across it).
  __device__ static int move_axis(int c, T &o, T v, int n) {
    if constexpr (G) {
      T x = o + v;
      if (x >= (T)n) {
        x -= (T)n;
      } else if (x < (T)0) {
        x += (T)n;
        if (x >= (T)n) x = (T)0;
      }
      o = x;
      if (!(x >= (T)0 && x < (T)n)) return -1;
      return (int)floor(x);
    } else {
      T x = o + v;
      if (x >= (T)1 || x < (T)0) {
        const T fl = floor(x);
        x -= fl;
        c += (int)fl;
        if (x >= (T)1) {
          x = (T)0;
          c += 1;
        }
      }
      o = x;
      return ((c % n) + n) % n;
    }
  }
};

// Records: set key and index, position and velocity from canonical FP64 input.
template <int P>
__global__ __launch_bounds__(BLOCK) void k3c_set_parts(const double *__restrict__ pos, const double *__restrict__ vel,
                                                       int n, Parts3<typename Prec<P>::T> pt,
                                                       Consts3<typename Prec<P>::T> k) {
  using T = typename Prec<P>::T;
  const int s = blockIdx.x * BLOCK + threadIdx.x;
  if (s >= n) return;
  const int nn[3] = {k.nx, k.ny, k.nz};
  int c[3];
  T o[3];
  bool ok = true;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const double X = pos[3 * s + q], fl = floor(X);
    ok = ok && fl >= 0.0 && fl < (double)nn[q];
    c[q] = ok ? (int)fl : 0;
    o[q] = Prec<P>::global_pos ? (T)X : (T)(X - fl);
    if (!Prec<P>::global_pos && o[q] >= (T)1) o[q] = (T)0.99999994f;  // float rounding to 1: keep in the cell
  }
  if (!ok) {  // reported; the particle is parked at the centre of cell 0
    atomicOr(&k.flags[FLAG_DOMAIN], 1);
    c[0] = c[1] = c[2] = 0;
    o[0] = o[1] = o[2] = (T)0.5;
  }
  pt.key[s] = (c[2] * k.ny + c[1]) * k.nx + c[0];
  pt.pid[s] = s;
  pt.px[s] = o[0];
  pt.py[s] = o[1];
  pt.pz[s] = o[2];
  pt.vx[s] = (T)vel[3 * s];
  pt.vy[s] = (T)vel[3 * s + 1];
  pt.vz[s] = (T)vel[3 * s + 2];
}

// The count of each particle's cell, with its arrival rank.
template <class T>
__global__ __launch_bounds__(BLOCK) void k3c_count(Parts3<T> pt, int n, int32_t *__restrict__ count,
                                                   int32_t *__restrict__ rank) {
  const int s = blockIdx.x * BLOCK + threadIdx.x;
  if (s < n) rank[s] = atomicAdd(&count[pt.key[s]], 1);
}

// Records to slot cs[key] + rank of the other set; slot of each index.
template <class T>
__global__ __launch_bounds__(BLOCK) void k3c_scatter(Parts3<T> src, Parts3<T> dst, const int32_t *__restrict__ rank,
                                                     const int32_t *__restrict__ cs, int n, int32_t *__restrict__ slot) {
  const int s = blockIdx.x * BLOCK + threadIdx.x;
  if (s >= n) return;
  const int key = src.key[s];
  const int d = cs[key] + rank[s];
  const int id = src.pid[s];
  dst.key[d] = key;
  dst.pid[d] = id;
  dst.px[d] = src.px[s];
  dst.py[d] = src.py[s];
  dst.pz[d] = src.pz[s];
  dst.vx[d] = src.vx[s];
  dst.vy[d] = src.vy[s];
  dst.vz[d] = src.vz[s];
  slot[id] = d;
}

// f^eq of Eq. 4 on D3Q19 (FP64, the oracle's operations in its order).
__device__ __forceinline__ double feq3_d(int i, double rho, double ux, double uy, double uz) {
  const double cu = (double)c3(i, 0) * ux + (double)c3(i, 1) * uy + (double)c3(i, 2) * uz;
  const double uu = ux * ux + uy * uy + uz * uz;
  return w3<double>(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
}
// Its deviation from w_i with FP32 arithmetic: w ((rho - 1) + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u)).
__device__ __forceinline__ float geq3_f(int i, float rho, float r1, float ux, float uy, float uz) {
  const float cu = (float)c3(i, 0) * ux + (float)c3(i, 1) * uy + (float)c3(i, 2) * uz;
  const float uu = ux * ux + uy * uy + uz * uz;
  return w3<float>(i) * (r1 + rho * (3.0f * cu + 4.5f * cu * cu - 1.5f * uu));
}

// ---------------------------------------------------------------- deposition + collision + streaming
// One thread per cell.  The cell's segment of the sorted records is put in
// ascending particle index (insertion sort of the records; the binning leaves
// arrival order), n and the velocity sum are taken in that order (Eq. 8),
// then the collision of Eq. 23, the force of Eq. 25, the velocities of Eq. 24
// and beta at the node, and the push to x + c_i.
template <int P>
__global__ __launch_bounds__(BLOCK) void k3c_collide(const typename Prec<P>::S *__restrict__ fsrc,
                                                     typename Prec<P>::S *__restrict__ fdst,
                                                     Fields3<typename Prec<P>::T> fl, const int32_t *__restrict__ cs,
                                                     Parts3<typename Prec<P>::T> pt,
                                                     const typename Prec<P>::T *__restrict__ lut,
                                                     Consts3<typename Prec<P>::T> k, int32_t *dg_n) {
  using T = typename Prec<P>::T;
  const int c = blockIdx.x * BLOCK + threadIdx.x;
  if (c >= k.C) return;
  const size_t C = (size_t)k.C;
  T f[Q3];
#pragma unroll
  for (int i = 0; i < Q3; ++i) f[i] = load_v<P>(fsrc, (size_t)i * C + c);
  const int a0 = cs[c], a1 = cs[c + 1], n = a1 - a0;
  for (int i = a0 + 1; i < a1; ++i) {  // insertion sort by particle index
    const int kv = pt.pid[i];
    if (pt.pid[i - 1] <= kv) continue;
    const T x0 = pt.px[i], y0 = pt.py[i], z0 = pt.pz[i], u0 = pt.vx[i], v0 = pt.vy[i], w0 = pt.vz[i];
    const int k0 = pt.key[i];
    int j = i - 1;
    do {
      pt.pid[j + 1] = pt.pid[j];
      pt.key[j + 1] = pt.key[j];
      pt.px[j + 1] = pt.px[j];
      pt.py[j + 1] = pt.py[j];
      pt.pz[j + 1] = pt.pz[j];
      pt.vx[j + 1] = pt.vx[j];
      pt.vy[j + 1] = pt.vy[j];
      pt.vz[j + 1] = pt.vz[j];
      --j;
    } while (j >= a0 && pt.pid[j] > kv);
    pt.pid[j + 1] = kv;
    pt.key[j + 1] = k0;
    pt.px[j + 1] = x0;
    pt.py[j + 1] = y0;
    pt.pz[j + 1] = z0;
    pt.vx[j + 1] = u0;
    pt.vy[j + 1] = v0;
    pt.vz[j + 1] = w0;
  }
  T vs[3] = {(T)0, (T)0, (T)0};
  for (int s = a0; s < a1; ++s) {
    vs[0] += pt.vx[s];
    vs[1] += pt.vy[s];
    vs[2] += pt.vz[s];
  }
  if (n > 0)
#pragma unroll
    for (int q = 0; q < 3; ++q) vs[q] = vs[q] / (T)n;
  const T *L = lut + (size_t)min(n, k.nlut - 1) * L3_W;
  const T relax = L[L3_RELAX], omg = L[L3_OMG], eg = L[L3_EG];
  T fs[Q3], F[3] = {(T)0, (T)0, (T)0}, j[3] = {(T)0, (T)0, (T)0}, rho_store;
  T rho;
  if constexpr (P == PREC_FP64) {
    T r = 0.0;
#pragma unroll
    for (int i = 0; i < Q3; ++i) {
      r += f[i];
#pragma unroll
      for (int q = 0; q < 3; ++q) j[q] += (T)c3(i, q) * f[i];
    }
    const T u[3] = {j[0] / r, j[1] / r, j[2] / r};
#pragma unroll
    for (int i = 0; i < Q3; ++i) {
      const int o = opp3(i);
      const T om = f[o] - f[i] + feq3_d(i, r, vs[0], vs[1], vs[2]) - feq3_d(o, r, u[0], u[1], u[2]);
      fs[i] = f[i] - relax * (f[i] - feq3_d(i, r, u[0], u[1], u[2])) + omg * om + k.src[i];
#pragma unroll
      for (int q = 0; q < 3; ++q) F[q] += (T)c3(i, q) * om;
    }
    rho = r;
    rho_store = r;
  } else {
    // deviations: rho - 1 = sum g, j = sum c g, and in Eq. 7 the weights of
    // f_opp(i) and f_i cancel
    T r1 = (T)0;
#pragma unroll
    for (int i = 0; i < Q3; ++i) {
      r1 += f[i];
#pragma unroll
      for (int q = 0; q < 3; ++q) j[q] += (T)c3(i, q) * f[i];
    }
    rho = (T)1 + r1;
    const T ir = dv<P>((T)1, rho);
    const T u[3] = {j[0] * ir, j[1] * ir, j[2] * ir};
#pragma unroll
    for (int i = 0; i < Q3; ++i) {
      const int o = opp3(i);
      const T om = f[o] - f[i] + geq3_f(i, rho, r1, vs[0], vs[1], vs[2]) - geq3_f(o, rho, r1, u[0], u[1], u[2]);
      fs[i] = f[i] - relax * (f[i] - geq3_f(i, rho, r1, u[0], u[1], u[2])) + omg * om + k.src[i];
#pragma unroll
      for (int q = 0; q < 3; ++q) F[q] += (T)c3(i, q) * om;
    }
    rho_store = r1;
  }
  T ug[3], sl2 = (T)0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    F[q] = omg * F[q];
    const T usup = dv<P>(j[q] + (T)0.5 * F[q] + k.halfG[q], rho);
    ug[q] = dv<P>(usup, eg);
    const T dd = ug[q] - vs[q];
    sl2 += dd * dd;
  }
  const T slip = sq<P>(sl2);
  T beta;
  if (L[L3_DILUTE] != (T)0) {
    const T re = dv<P>(L[L3_BRE] * slip * k.d, k.mu);
    if (re < (T)1000)
      beta = L[L3_A] * ((T)1.0 + (T)0.15 * pw<P>(re, (T)0.687));
    else
      beta = dv<P>(L[L3_H] * slip * (T)0.44 * L[L3_OM], k.d);
  } else {
    beta = L[L3_D1] + dv<P>(L[L3_D2] * slip, k.d);
  }
  fl.rho[c] = rho_store;
  fl.ugx[c] = ug[0];
  fl.ugy[c] = ug[1];
  fl.ugz[c] = ug[2];
  fl.fpx[c] = F[0];
  fl.fpy[c] = F[1];
  fl.fpz[c] = F[2];
  fl.beta[c] = beta;
  fl.es[c] = L[L3_ES];
  if (dg_n) dg_n[c] = n;
  int x, y, z;
  cell3_xyz(k, c, x, y, z);
#pragma unroll
  for (int i = 0; i < Q3; ++i) {
    const int tx = wrap_p(x + c3(i, 0), k.nx), ty = wrap_p(y + c3(i, 1), k.ny), tz = wrap_p(z + c3(i, 2), k.nz);
    store_v<P>(fdst, (size_t)i * C + ((size_t)tz * k.ny + ty) * k.nx + tx, fs[i]);
  }
}

// Node pressure gradient (central differences of p = rho / 3, periodic),
// packed with the node's u_gas, solid fraction and beta for the interpolation.
template <int P>
__global__ __launch_bounds__(BLOCK) void k3c_gradp(Fields3<typename Prec<P>::T> fl, Consts3<typename Prec<P>::T> k) {
  using T = typename Prec<P>::T;
  const int c = xcd_block<XCD_RUN_3D_GRADP>(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
  if (c >= k.C) return;
  int x, y, z;
  cell3_xyz(k, c, x, y, z);
  const int nxy = k.nx * k.ny;
  const int xp = z * nxy + y * k.nx + wrap_p(x + 1, k.nx), xm = z * nxy + y * k.nx + wrap_p(x - 1, k.nx);
  const int yp = z * nxy + wrap_p(y + 1, k.ny) * k.nx + x, ym = z * nxy + wrap_p(y - 1, k.ny) * k.nx + x;
  const int zp = wrap_p(z + 1, k.nz) * nxy + y * k.nx + x, zm = wrap_p(z - 1, k.nz) * nxy + y * k.nx + x;
  Node8<T> nd;
  nd.v[0] = fl.ugx[c];
  nd.v[1] = fl.ugy[c];
  nd.v[2] = fl.ugz[c];
  nd.v[3] = fl.es[c];
  nd.v[4] = fl.beta[c];
  nd.v[5] = (dv<P>(fl.rho[xp], (T)3.0) - dv<P>(fl.rho[xm], (T)3.0)) * (T)0.5;
  nd.v[6] = (dv<P>(fl.rho[yp], (T)3.0) - dv<P>(fl.rho[ym], (T)3.0)) * (T)0.5;
  nd.v[7] = (dv<P>(fl.rho[zp], (T)3.0) - dv<P>(fl.rho[zm], (T)3.0)) * (T)0.5;
  reinterpret_cast<Node8<T> *>(fl.node)[c] = nd;
}

// Gas quantities at one particle: trilinear interpolation of u_gas, the solid
// fraction, beta and grad p from the 8 nodes around it (nodes at the cell
// centres, periodic), in the oracle's order of nodes and products.
template <int P> struct Interp3 {
  using T = typename Prec<P>::T;
  T u[3], es, beta, gp[3];
  __device__ void at(const Consts3<T> &k, const Fields3<T> &fl, const int *cc, const T *o) {
    int i0[3];
    T t[3];
    const int nn[3] = {k.nx, k.ny, k.nz};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      Pos3<P>::axis_stencil(cc[q], o[q], i0[q], t[q]);
      i0[q] = min(max(i0[q], -1), nn[q] - 1);  // a position in the box needs no clamp; a NaN stays in bounds
    }
    u[0] = u[1] = u[2] = es = beta = gp[0] = gp[1] = gp[2] = (T)0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int ox = q & 1, oy = (q >> 1) & 1, oz = q >> 2;
      const int id = (wrap_p(i0[2] + oz, k.nz) * k.ny + wrap_p(i0[1] + oy, k.ny)) * k.nx + wrap_p(i0[0] + ox, k.nx);
      const T w = (ox ? t[0] : (T)1.0 - t[0]) * (oy ? t[1] : (T)1.0 - t[1]) * (oz ? t[2] : (T)1.0 - t[2]);
      const Node8<T> nd = reinterpret_cast<const Node8<T> *>(fl.node)[id];
      u[0] += w * nd.v[0];
      u[1] += w * nd.v[1];
      u[2] += w * nd.v[2];
      es += w * nd.v[3];
      beta += w * nd.v[4];
      gp[0] += w * nd.v[5];
      gp[1] += w * nd.v[6];
      gp[2] += w * nd.v[7];
    }
  }
};

// ---------------------------------------------------------------- drag, integration, binning count
// One thread per particle slot (a cell-per-thread form left most lanes idle:
// about one cell in seven holds a sphere).  Each thread interpolates at its
// particle and keeps its pre-estimated drag (Eq. 26) in LDS; then it sums the
// pre-drags of its cell's segment in slot order (ascending index, as the
// collide kernel left it) for Eq. 27, taking members outside the workgroup's
// slots (only the first and last cell of a workgroup can have them) from the
// same interpolation done again, applies Eq. 28 and the acceleration of
// Eq. 16, moves the particle with the periodic wrap and counts it into its
// new cell.  The moved record goes to the same slot of the other record set
// (out), so the records every workgroup reads stay as they were.  Six waves
// per SIMD (68 VGPRs in FP32) rather than the five the registers allow
// unbounded: 1.5 % faster; eight were 6.5 % slower.
template <int P> struct PreDrag3 {
  using T = typename Prec<P>::T;
  T pd[3];  // cf (u_gas - v), Eq. 26 before the per-cell correction
  Interp3<P> I;
  __device__ void at(const Parts3<T> &pt, const Fields3<T> &fl, const Consts3<T> &k, int t) {
    int cc[3];
    cell3_xyz(k, pt.key[t], cc[0], cc[1], cc[2]);
    const T o[3] = {pt.px[t], pt.py[t], pt.pz[t]}, v[3] = {pt.vx[t], pt.vy[t], pt.vz[t]};
    I.at(k, fl, cc, o);
    const T cf = dv<P>(k.vp * I.beta, I.es);
#pragma unroll
    for (int q = 0; q < 3; ++q) pd[q] = cf * (I.u[q] - v[q]);
  }
};

template <int P>
__global__ __launch_bounds__(BLOCK) LBDPS_WAVES6 void k3c_drag(Parts3<typename Prec<P>::T> pt, Parts3<typename Prec<P>::T> out,
                                                  Fields3<typename Prec<P>::T> fl, const int32_t *__restrict__ cs,
                                                  Consts3<typename Prec<P>::T> k, int32_t *__restrict__ count,
                                                  int32_t *__restrict__ rank, typename Prec<P>::T *dg_fd,
                                                  typename Prec<P>::T *dg_acc) {
  using T = typename Prec<P>::T;
  __shared__ T spd[3][BLOCK];
  const int s0 = blockIdx.x * BLOCK, s = s0 + threadIdx.x, s1 = min(s0 + BLOCK, k.npart);
  PreDrag3<P> me;
  if (s < k.npart) {
    me.at(pt, fl, k, s);
#pragma unroll
    for (int q = 0; q < 3; ++q) spd[q][threadIdx.x] = me.pd[q];
  }
  __syncthreads();
  if (s >= k.npart) return;
  const int c = pt.key[s];
  const int a0 = cs[c], a1 = cs[c + 1], n = a1 - a0;
  T S[3] = {(T)0, (T)0, (T)0};
  for (int t = a0; t < a1; ++t) {
    T pd[3];
    if (t >= s0 && t < s1) {
#pragma unroll
      for (int q = 0; q < 3; ++q) pd[q] = spd[q][t - s0];
    } else {  // a member held by the neighbouring workgroup
      PreDrag3<P> o;
      o.at(pt, fl, k, t);
#pragma unroll
      for (int q = 0; q < 3; ++q) pd[q] = o.pd[q];
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) S[q] += pd[q];
  }
  int cc[3];
  cell3_xyz(k, c, cc[0], cc[1], cc[2]);
  const T fg[3] = {fl.fpx[c], fl.fpy[c], fl.fpz[c]};
  const int nn[3] = {k.nx, k.ny, k.nz};
  T o[3] = {pt.px[s], pt.py[s], pt.pz[s]}, v[3] = {pt.vx[s], pt.vy[s], pt.vz[s]};
  int nc[3];
  T fd[3], acc[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const T pr = me.pd[q];
    fd[q] = S[q] == (T)0 ? dv<P>(-fg[q], (T)n) : dv<P>(-fg[q] * pr, S[q]);
    acc[q] = k.geff[q] + dv<P>(fd[q] + k.fp * me.I.gp[q], k.m);
    v[q] = v[q] + acc[q];
    nc[q] = Pos3<P>::move_axis(cc[q], o[q], v[q], nn[q]);
  }
  const int id = pt.pid[s];
  if (dg_fd) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      dg_fd[3 * (size_t)id + q] = fd[q];
      dg_acc[3 * (size_t)id + q] = acc[q];
    }
  }
  int nk = (nc[2] * k.ny + nc[1]) * k.nx + nc[0];
  if (nc[0] < 0 || nc[1] < 0 || nc[2] < 0) {  // not a position in the box: reported, counted in its old cell
    atomicOr(&k.flags[FLAG_DOMAIN], 1);
    nk = c;
  }
  out.key[s] = nk;
  out.pid[s] = id;
  out.px[s] = o[0];
  out.py[s] = o[1];
  out.pz[s] = o[2];
  out.vx[s] = v[0];
  out.vy[s] = v[1];
  out.vz[s] = v[2];
  rank[s] = atomicAdd(&count[nk], 1);
}

// ---------------------------------------------------------------- contacts
// One thread per particle slot.  A partner lies within d < 1, so only the
// cells that come within d of the particle along each axis can hold one (two
// of the three per axis for d <= 1/2, with a rounding margin).  Contacts are
// kept as a row sorted by particle index (index << 32 | slot), as in 2-D.
// Eight waves per SIMD (58 VGPRs in FP32, no spill) instead of seven: the
// search is a chain of dependent loads, and the extra wave makes it 10 %
// faster on the 256 x 256 x 1024 riser.
template <int P>
__global__ __launch_bounds__(BLOCK) LBDPS_WAVES8 void k3c_contacts(Parts3<typename Prec<P>::T> pt, const int32_t *__restrict__ cs,
                                                      Consts3<typename Prec<P>::T> k, Adj adj,
                                                      int32_t *__restrict__ deg, int32_t *__restrict__ done,
                                                      int32_t *ticket, int32_t *__restrict__ chunk_busy,
                                                      long long *pair_part, int32_t *need_sweep,
                                                      long long *__restrict__ roots, int32_t *__restrict__ rcount) {
  using T = typename Prec<P>::T;
  __shared__ long long sh[BLOCK / 64];
  __shared__ int shi[BLOCK / 64];
  const int bidx = xcd_block<XCD_RUN_3D_CONTACTS>(blockIdx.x, gridDim.x);  // the tile, and the index of its list
  const int s = bidx * BLOCK + threadIdx.x;
  if (s == 0) {
    *ticket = 0;
    *need_sweep = 0;
  }
  long long fwd = 0;
  bool cand = false;  // has contacts, all with higher indices: a possible cluster root
  if (s < k.npart) {
    const int key = pt.key[s], id = pt.pid[s];
    const T a[3] = {pt.px[s], pt.py[s], pt.pz[s]};
    int cc[3];
    cell3_xyz(k, key, cc[0], cc[1], cc[2]);
    const int nn[3] = {k.nx, k.ny, k.nz};
    // the axis offsets (-1, 0, +1) whose cells come within d of the particle
    bool use[3][3];
    const T margin = (T)1e-5;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const T fr = Prec<P>::global_pos ? a[q] - (T)cc[q] : a[q];
      use[q][0] = fr < k.d + margin;
      use[q][1] = true;
      use[q][2] = fr > (T)1 - k.d - margin;
    }
    const AdjRow row = adj.row(s);
    int cnt = 0;
    bool over = false;
    auto test = [&](int t) {
      if (t == s) return;
      const T b[3] = {pt.px[t], pt.py[t], pt.pz[t]};
      T d[3];
      Pos3<P>::sep(k, key, a, pt.key[t], b, d);
      if (!(d[0] * d[0] + d[1] * d[1] + d[2] * d[2] <= k.dd)) return;
      const int tid = pt.pid[t];
      if (tid > id) ++fwd;
      if (cnt == KMAX) {
        over = true;
        return;
      }
      const long long e = ((long long)tid << 32) | (unsigned)t;
      int j = cnt;
      while (j > 0 && row[j - 1] > e) {
        row[j] = row[j - 1];
        --j;
      }
      row[j] = e;
      ++cnt;
    };
    // The cells of one (y, z) row next to each other in x are one slot range:
    // away from the x seam, the bounds of all (at most nine) ranges are read
    // together, then their candidates tested.
    const bool xin = (!use[0][0] || cc[0] >= 1) && (!use[0][2] || cc[0] <= k.nx - 2);
    if (xin) {
      int lo[9], hi[9];
#pragma unroll
      for (int r = 0; r < 9; ++r) {
        const int oz = r / 3 - 1, oy = r % 3 - 1;
        lo[r] = hi[r] = 0;
        if (use[2][oz + 1] && use[1][oy + 1]) {
          const int base = (wrap_p(cc[2] + oz, nn[2]) * k.ny + wrap_p(cc[1] + oy, nn[1])) * k.nx;
          lo[r] = cs[base + cc[0] - (use[0][0] ? 1 : 0)];
          hi[r] = cs[base + cc[0] + 1 + (use[0][2] ? 1 : 0)];
        }
      }
#pragma unroll
      for (int r = 0; r < 9; ++r)
        for (int t = lo[r]; t < hi[r]; ++t) test(t);
    } else {
      for (int oz = -1; oz <= 1; ++oz) {
        if (!use[2][oz + 1]) continue;
        for (int oy = -1; oy <= 1; ++oy) {
          if (!use[1][oy + 1]) continue;
          for (int ox = -1; ox <= 1; ++ox) {
            if (!use[0][ox + 1]) continue;
            const int nb =
                (wrap_p(cc[2] + oz, nn[2]) * k.ny + wrap_p(cc[1] + oy, nn[1])) * k.nx + wrap_p(cc[0] + ox, nn[0]);
            for (int t = cs[nb]; t < cs[nb + 1]; ++t) test(t);
          }
        }
      }
    }
    if (over) atomicOr(&k.flags[FLAG_CAPACITY], 1);
    deg[s] = cnt;
    done[s] = 0;
    if (cnt > 0) {
      chunk_busy[id / RES_CHUNK] = 1;
      cand = (int)(row[0] >> 32) > id;
    }
  }
  // candidate roots of this workgroup, compacted to the front of its segment
  int nc;
  const int off = block_excl_scan(cand ? 1 : 0, shi, nc);
  if (cand) roots[(size_t)bidx * BLOCK + off] = ((long long)pt.pid[s] << 32) | (unsigned)s;
  const long long t = block_sum_ll(fwd, sh);
  if (threadIdx.x == 0) {
    pair_part[bidx] = t;
    rcount[bidx] = nc;
  }
}

// ---------------------------------------------------------------- contact clusters
// As in 2-D: a lane takes a candidate root, gathers its cluster (the contact
// kernel's rows, up to CL_LDS members, giving up at a lower index), orders the
// members by index and applies the cluster's pairs in lexicographic order,
// which is the sequential sweep's result bit for bit (clusters touch disjoint
// particles).  A member loads its record and up to NB3 higher neighbours' in
// one round.  A cluster of more members is left to the ordered sweep.
template <int P, class Row>
__device__ __forceinline__ void resolve_cluster3(Row q, int m, unsigned long long A,
                                                 const Consts3<typename Prec<P>::T> &k,
                                                 Parts3<typename Prec<P>::T> &pt, int32_t *done, long long &ncoll) {
  using T = typename Prec<P>::T;
  constexpr int NB3 = 2;
  sort_members(q, m);
  for (int i = 0; i < m; ++i) {
    const long long qi = q[i];
    const int u = (int)(qi & 0x1fffffffll);
    const unsigned nbr = (unsigned)(A >> (8 * (int)((qi >> 29) & 7))) & 0xffu;  // places of u's neighbours
    const int ku = ldu(pt.key, u);
    const T a[3] = {ldu(pt.px, u), ldu(pt.py, u), ldu(pt.pz, u)};
    T vu[3] = {ldu(pt.vx, u), ldu(pt.vy, u), ldu(pt.vz, u)};
    int j = i + 1;  // next member (in index order) to look at
    while (true) {
      int w[NB3], kw[NB3];
      T b[NB3][3], vw[NB3][3];
      int nw = 0;
      for (; j < m && nw < NB3; ++j) {
        const long long qj = q[j];
        if (nbr >> (int)((qj >> 29) & 7) & 1u) {
#pragma unroll
          for (int c = 0; c < NB3; ++c)
            if (c == nw) w[c] = (int)(qj & 0x1fffffffll);
          ++nw;
        }
      }
#pragma unroll
      for (int c = 0; c < NB3; ++c)
        if (c < nw) {
          kw[c] = ldu(pt.key, w[c]);
          b[c][0] = ldu(pt.px, w[c]);
          b[c][1] = ldu(pt.py, w[c]);
          b[c][2] = ldu(pt.pz, w[c]);
          vw[c][0] = ldu(pt.vx, w[c]);
          vw[c][1] = ldu(pt.vy, w[c]);
          vw[c][2] = ldu(pt.vz, w[c]);
        }
#pragma unroll
      for (int c = 0; c < NB3; ++c)
        if (c < nw) {
          T d[3];
          Pos3<P>::sep(k, ku, a, kw[c], b[c], d);
          const T dot = (vu[0] - vw[c][0]) * d[0] + (vu[1] - vw[c][1]) * d[1] + (vu[2] - vw[c][2]) * d[2];
          if (dot < (T)0) {
            const T r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            const T q0 = (k.one_e * dot) / r2;
            const T ci = (q0 * k.m) / k.msum;
#pragma unroll
            for (int e = 0; e < 3; ++e) {
              vu[e] = vu[e] - ci * d[e];
              vw[c][e] = vw[c][e] + ci * d[e];
            }
            pt.vx[w[c]] = vw[c][0];
            pt.vy[w[c]] = vw[c][1];
            pt.vz[w[c]] = vw[c][2];
            ++ncoll;
          }
        }
      if (j >= m) break;
    }
    pt.vx[u] = vu[0];
    pt.vy[u] = vu[1];
    pt.vz[u] = vu[2];
    done[u] = __builtin_popcount(nbr) | DONE_WHOLE;  // its contacts, all inside the cluster
  }
}

constexpr int RC3_LISTS = 4;  // candidate lists per cluster workgroup

template <int P>
__global__ __launch_bounds__(BLOCK) void k3c_clusters(Parts3<typename Prec<P>::T> pt, Adj adj,
                                                      const int32_t *__restrict__ deg, int32_t *done,
                                                      Consts3<typename Prec<P>::T> k, int32_t *need_sweep,
                                                      long long *coll_part, const long long *__restrict__ roots,
                                                      const int32_t *__restrict__ rcount, int nlists) {
  __shared__ long long sh[BLOCK / 64];
  __shared__ int shi[BLOCK / 64];
  __shared__ int pre[BLOCK + 1];
  __shared__ long long qs[CL_LDS * BLOCK];
  const int bidx = blockIdx.x, gdim = gridDim.x;
  const int per = (nlists + gdim - 1) / gdim;  // <= BLOCK (host grid choice)
  const int b0 = bidx * per;
  const int nb = max(0, min(nlists - b0, per));
  // a contact row over its capacity leaves the contact graph incomplete
  const bool overflow = __hip_atomic_load(&k.flags[FLAG_CAPACITY], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
  const int c = (!overflow && (int)threadIdx.x < nb) ? rcount[b0 + threadIdx.x] : 0;
  int tot;
  const int o = block_excl_scan(c, shi, tot);
  long long ncoll = 0;
  if (tot > 0) {  // uniform
    if ((int)threadIdx.x < nb) pre[threadIdx.x] = o;
    if (threadIdx.x == 0) pre[nb] = tot;
    __syncthreads();
    const LdsColumn ql{qs + threadIdx.x};
    for (int f = threadIdx.x; f < tot; f += BLOCK) {
      int lo = 0, hi = nb;  // list j with pre[j] <= f < pre[j + 1]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= f) lo = mid;
        else hi = mid;
      }
      const long long r = roots[(size_t)(b0 + lo) * BLOCK + (f - pre[lo])];
      const int s = (int)(r & 0xffffffffll), g = (int)(r >> 32);
      unsigned long long A;
      const int m = gather_cluster(ql, CL_LDS, s, g, adj, deg, A);
      if (m > 0) resolve_cluster3<P>(ql, m, A, k, pt, done, ncoll);
      else if (m < 0) atomicOr(need_sweep, 1);  // too large: the ordered sweep takes it
    }
  }
  const long long tc = block_sum_ll(ncoll, sh);
  if (threadIdx.x == 0) coll_part[bidx] = tc;
}

// ---------------------------------------------------------------- collision resolution (Eqs. 17-18)
// Pairs (i, j), i < j, in lexicographic order with the current velocities,
// as an ordered sweep: chunks of RES_CHUNK particle indices in increasing
// order from an atomic ticket; a lane owns indices base + j BLOCK and fires a
// pair once both particles have finished every earlier pair (done counts),
// so each particle's pairs run in its row's order and the result is the
// sequential sweep's bit for bit.  The owner of the earliest unfinished pair
// is always running, so the sweep progresses; waits are bounded by
// spin_limit polls (FLAG_STALL past it).  A contact row over its capacity
// leaves the graph incomplete: the sweep is skipped.
template <int P>
__device__ __forceinline__ bool pair3(const Consts3<typename Prec<P>::T> &k, Parts3<typename Prec<P>::T> &pt, int s,
                                      int t) {
  using T = typename Prec<P>::T;
  const T a[3] = {pt.px[s], pt.py[s], pt.pz[s]}, b[3] = {pt.px[t], pt.py[t], pt.pz[t]};
  T d[3];
  Pos3<P>::sep(k, pt.key[s], a, pt.key[t], b, d);
  T vi[3] = {pt.vx[s], pt.vy[s], pt.vz[s]}, vj[3] = {pt.vx[t], pt.vy[t], pt.vz[t]};
  const T dot = (vi[0] - vj[0]) * d[0] + (vi[1] - vj[1]) * d[1] + (vi[2] - vj[2]) * d[2];
  if (!(dot < (T)0)) return false;
  const T r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  const T q0 = (k.one_e * dot) / r2;
  const T ci = (q0 * k.m) / k.msum;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    vi[q] = vi[q] - ci * d[q];
    vj[q] = vj[q] + ci * d[q];
  }
  pt.vx[s] = vi[0];
  pt.vy[s] = vi[1];
  pt.vz[s] = vi[2];
  pt.vx[t] = vj[0];
  pt.vy[t] = vj[1];
  pt.vz[t] = vj[2];
  return true;
}

template <int P>
__global__ __launch_bounds__(BLOCK) void k3c_resolve(Parts3<typename Prec<P>::T> pt, const int32_t *__restrict__ slot,
                                                     Adj adj, const int32_t *__restrict__ deg, int32_t *done,
                                                     int32_t *ticket, Consts3<typename Prec<P>::T> k,
                                                     long long *coll_part, int32_t *__restrict__ chunk_busy,
                                                     const int32_t *need_sweep) {
  __shared__ int s_ticket;
  __shared__ long long sh[BLOCK / 64];
  long long ncoll = 0;
  unsigned spins = 0;
  const int nchunks = (k.npart + RES_CHUNK - 1) / RES_CHUNK;
  // every cluster was resolved whole, or a contact row overflowed (the
  // resolution is skipped): only clear the chunk marks
  if (!*need_sweep || __hip_atomic_load(&k.flags[FLAG_CAPACITY], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < nchunks; i += gridDim.x * BLOCK) chunk_busy[i] = 0;
    if (threadIdx.x == 0) coll_part[blockIdx.x] = 0;
    return;
  }
  for (;;) {
    if (threadIdx.x == 0) {
      int tk;
      do {
        tk = atomicAdd(ticket, 1);
      } while (tk < nchunks && chunk_busy[tk] == 0);
      s_ticket = tk;
    }
    __syncthreads();
    const int tk = s_ticket;
    __syncthreads();
    if (tk >= nchunks) break;
    if (threadIdx.x == 0) chunk_busy[tk] = 0;
    const int base = tk * RES_CHUNK + (int)threadIdx.x;
    int j = 0, g = base;
    int state = 2;  // 0: pair pending, 1: finished this particle's pairs, 2: lane done
    int s = 0, dg = 0, a = 0, t = 0, b = 0;
    AdjRow row{nullptr, nullptr};
    auto next = [&]() {
      for (; j < RES_ITEMS; ++j) {
        g = base + j * BLOCK;
        if (g >= k.npart) {
          j = RES_ITEMS;
          break;
        }
        s = slot[g];
        dg = deg[s];
        if (dg == 0 || done[s] >= DONE_WHOLE) continue;  // no contacts (fully periodic: no wall pass), or resolved whole
        row = adj.row(s);
        a = 0;
        while (a < dg && (int)(row[a] >> 32) < g) ++a;
        if (a < dg) {
          t = (int)(row[a] & 0xffffffffll);
          b = row_position(adj, deg, t, g);
          state = 0;
        } else {
          state = 1;
        }
        return;
      }
      state = 2;
    };
    next();
    while (__any(state != 2)) {
      bool progressed = false;
      if (state == 0) {
        const int ds = __hip_atomic_load(&done[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int dt = __hip_atomic_load(&done[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (ds == a && dt == b) {
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          ncoll += pair3<P>(k, pt, s, t);
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          __hip_atomic_store(&done[t], b + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(&done[s], a + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ++a;
          if (a < dg) {
            t = (int)(row[a] & 0xffffffffll);
            b = row_position(adj, deg, t, g);
          } else {
            state = 1;
          }
          progressed = true;
        }
      } else if (state == 1) {
        const int ds = __hip_atomic_load(&done[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (ds == dg) {
          ++j;
          next();
          progressed = true;
        }
      }
      if (state != 2 && !progressed) {
        if (++spins > k.spin_limit) {
          atomicOr(&k.flags[FLAG_STALL], 1);
          state = 2;
          j = RES_ITEMS;
        } else {
          __builtin_amdgcn_s_sleep(1);
        }
      }
    }
  }
  const long long tc = block_sum_ll(ncoll, sh);
  if (threadIdx.x == 0) coll_part[blockIdx.x] = tc;
}

// ---------------------------------------------------------------- canonical FP64 state in and out
// Populations [19][nz][ny][nx] from FP64 (NULL: f^eq(1, 0) = w_i), stored as
// values (FP64) or as deviations f_i - w_i rounded to the storage type.
template <int P>
__global__ __launch_bounds__(BLOCK) void k3_set_f(const double *__restrict__ fin, typename Prec<P>::S *__restrict__ f,
                                                  int C) {
  using T = typename Prec<P>::T;
  const long long e = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (e >= (long long)Q3 * C) return;
  const int i = (int)(e / C);
  const double v = fin ? fin[e] : w3<double>(i);
  if constexpr (P == PREC_FP64) f[e] = v;
  else store_v<P>(f, (size_t)e, (T)(v - w3<double>(i)));
}

template <int P>
__global__ __launch_bounds__(BLOCK) void k3_get_f(const typename Prec<P>::S *__restrict__ f, double *__restrict__ out,
                                                  int C) {
  const long long e = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (e >= (long long)Q3 * C) return;
  if constexpr (P == PREC_FP64) out[e] = f[e];
  else out[e] = w3<double>((int)(e / C)) + (double)load_v<P>(f, (size_t)e);
}

// ---------------------------------------------------------------- FP64 conservation sums (fixed-order reductions)
// Per workgroup over a fixed stride of cells: the mass and gas momentum of the
// canonical populations (the weights plus the deviations in the reduced
// storages), part[4 b + j]; a non-finite value sets *nonfinite.
template <int P>
__global__ __launch_bounds__(BLOCK) void k3_cons_cells(const typename Prec<P>::S *__restrict__ f, long long C,
                                                       double *__restrict__ part, int32_t *nonfinite) {
  __shared__ double sh[BLOCK / 64];
  double m = 0.0, q[3] = {0.0, 0.0, 0.0};
  int bad = 0;
  for (long long c = (long long)blockIdx.x * BLOCK + threadIdx.x; c < C; c += (long long)gridDim.x * BLOCK) {
#pragma unroll
    for (int i = 0; i < Q3; ++i) {
      double v;
      if constexpr (P == PREC_FP64) v = f[(size_t)i * C + c];
      else v = w3<double>(i) + (double)load_v<P>(f, (size_t)i * C + c);
      bad |= !isfinite(v);
      m += v;
#pragma unroll
      for (int a = 0; a < 3; ++a) q[a] += (double)c3(i, a) * v;
    }
  }
  if (bad) atomicOr(nonfinite, 1);
  const double t0 = block_sum_d(m, sh), t1 = block_sum_d(q[0], sh), t2 = block_sum_d(q[1], sh),
               t3 = block_sum_d(q[2], sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x * 4 + 0] = t0;
    part[blockIdx.x * 4 + 1] = t1;
    part[blockIdx.x * 4 + 2] = t2;
    part[blockIdx.x * 4 + 3] = t3;
  }
}

// The particles' momentum m v per workgroup, part[3 b + a].
template <class T>
__global__ __launch_bounds__(BLOCK) void k3_cons_parts(Parts3<T> pt, int n, double mass, double *__restrict__ part,
                                                       int32_t *nonfinite) {
  __shared__ double sh[BLOCK / 64];
  double q[3] = {0.0, 0.0, 0.0};
  int bad = 0;
  for (int s = blockIdx.x * BLOCK + threadIdx.x; s < n; s += gridDim.x * BLOCK) {
    const double v[3] = {(double)pt.vx[s], (double)pt.vy[s], (double)pt.vz[s]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      bad |= !isfinite(v[a]);
      q[a] += mass * v[a];
    }
  }
  if (bad) atomicOr(nonfinite, 1);
  const double t0 = block_sum_d(q[0], sh), t1 = block_sum_d(q[1], sh), t2 = block_sum_d(q[2], sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x * 3 + 0] = t0;
    part[blockIdx.x * 3 + 1] = t1;
    part[blockIdx.x * 3 + 2] = t2;
  }
}

// out[0] mass, out[1..3] gas momentum, out[4..6] particle momentum, out[7]
// 1 if a value was not finite: the workgroup partials summed in a fixed order.
__global__ __launch_bounds__(BLOCK) void k3_cons_final(const double *__restrict__ pc, int nbc,
                                                       const double *__restrict__ pp, int nbp,
                                                       const int32_t *nonfinite, double *out) {
  __shared__ double sh[BLOCK / 64];
  double v[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nbc; b += BLOCK)
    for (int j = 0; j < 4; ++j) v[j] += pc[b * 4 + j];
  for (int b = threadIdx.x; b < nbp; b += BLOCK)
    for (int j = 0; j < 3; ++j) v[4 + j] += pp[b * 3 + j];
  for (int j = 0; j < 7; ++j) {
    const double t = block_sum_d(v[j], sh);
    if (threadIdx.x == 0) out[j] = t;
  }
  if (threadIdx.x == 0) out[7] = *nonfinite ? 1.0 : 0.0;
}

// A field to FP64: one plane (out[i] = add + a[i]) or three interleaved
// (out[3 i + q] = plane q).
template <class T>
__global__ __launch_bounds__(BLOCK) void k3_get_field(const T *__restrict__ a, const T *__restrict__ b,
                                                      const T *__restrict__ c, long long n, double *out, double add) {
  const long long i = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= n) return;
  if (b) {
    out[3 * i] = (double)a[i];
    out[3 * i + 1] = (double)b[i];
    out[3 * i + 2] = (double)c[i];
  } else {
    out[i] = add + (double)a[i];
  }
}

// ---------------------------------------------------------------- canonical FP64 readouts
template <int P>
__global__ __launch_bounds__(BLOCK) void k3c_get_parts(Parts3<typename Prec<P>::T> pt, const int32_t *__restrict__ slot,
                                                       int n, Consts3<typename Prec<P>::T> k, double *pos,
                                                       double *vel) {
  const int id = blockIdx.x * BLOCK + threadIdx.x;
  if (id >= n) return;
  const int s = slot[id];
  int cc[3];
  cell3_xyz(k, pt.key[s], cc[0], cc[1], cc[2]);
  const double o[3] = {(double)pt.px[s], (double)pt.py[s], (double)pt.pz[s]};
  if (pos)
#pragma unroll
    for (int q = 0; q < 3; ++q) pos[3 * id + q] = Prec<P>::global_pos ? o[q] : (double)cc[q] + o[q];
  if (vel) {
    vel[3 * id] = (double)pt.vx[s];
    vel[3 * id + 1] = (double)pt.vy[s];
    vel[3 * id + 2] = (double)pt.vz[s];
  }
}

}  // namespace lbdps
