// HIP kernels of one coupled step (gfx950, wave64).  Citations name the
// equation or section of Wang, Zhang, Wang, Ge & Li, "Lattice Boltzmann based
// discrete simulation for gas-solid fluidization" that each piece computes.
//
// Arithmetic order: in FP64 every expression is written in the order the
// method's reference formulation evaluates it, and the library is compiled
// with contraction off, so FP64 results agree with an FP64 evaluation of the
// same formulas to the last bit except where pow() is involved.
#pragma once

#include "device.hpp"

namespace lbdps {

// ------------------------------------------------------------------ helpers
template <class T>
__device__ __forceinline__ T feq(int i, T rho, T ux, T uy) {
  // Eq. 4 with c_s^2 = 1/3.
  T cu = (T)cx_of(i) * ux + (T)cy_of(i) * uy;
  T uu = ux * ux + uy * uy;
  return wgt<T>(i) * rho * ((T)1.0 + (T)3.0 * cu + (T)4.5 * cu * cu - (T)1.5 * uu);
}

// Equilibrium in the stored form: f^eq_i (FP64), or f^eq_i - w_i =
// w_i ((rho - 1) + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u)) in the deviation modes.
template <int P>
__device__ __forceinline__ typename Prec<P>::T feq_v(int i, typename Prec<P>::T rho, typename Prec<P>::T rho1,
                                                     typename Prec<P>::T ux, typename Prec<P>::T uy) {
  using T = typename Prec<P>::T;
  if constexpr (kDev<P>) {
    T cu = (T)cx_of(i) * ux + (T)cy_of(i) * uy;
    T uu = ux * ux + uy * uy;
    return wgt<T>(i) * (rho1 + rho * ((T)3.0 * cu + (T)4.5 * cu * cu - (T)1.5 * uu));
  } else {
    return feq<T>(i, rho, ux, uy);
  }
}

__device__ __forceinline__ int wrap_i(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Node index for interpolation and gradients: wrap on periodic axes, clamp
// otherwise (node (i, j) sits at the cell centre (i + 1/2, j + 1/2)).  For
// i >= -n; the remainder is taken only beyond 2n (lattices narrower than a
// drag tile).
__device__ __forceinline__ int node_idx(int i, int n, int per) {
  if (!per) return i < 0 ? 0 : (i >= n ? n - 1 : i);
  if (i < 0) return i + n;
  return i < n ? i : (i - n < n ? i - n : i % n);
}

template <int P> struct Pos {
  using T = typename Prec<P>::T;
  static constexpr bool G = Prec<P>::global_pos;

  // Minimum-image separation a - b.
  __device__ static void sep(const Consts<T> &k, int ka, T xa, T ya, int kb, T xb, T yb, T &dx, T &dy) {
    if constexpr (G) {
      T x = xa - xb, y = ya - yb;
      if (k.per_x) {
        if (x > (T)0.5 * (T)k.nx)
          x -= (T)k.nx;
        else if (x < -(T)0.5 * (T)k.nx)
          x += (T)k.nx;
      }
      if (k.per_y) {
        if (y > (T)0.5 * (T)k.ny)
          y -= (T)k.ny;
        else if (y < -(T)0.5 * (T)k.ny)
          y += (T)k.ny;
      }
      dx = x;
      dy = y;
    } else {
      int ax, ay, bx, by;
      cell_xy(k, ka, ax, ay);
      cell_xy(k, kb, bx, by);
      int dcx = ax - bx, dcy = ay - by;
      if (k.per_x) {
        if (dcx > k.nx / 2)
          dcx -= k.nx;
        else if (dcx < -(k.nx / 2))
          dcx += k.nx;
      }
      if (k.per_y) {
        if (dcy > k.ny / 2)
          dcy -= k.ny;
        else if (dcy < -(k.ny / 2))
          dcy += k.ny;
      }
      T ox = xa - xb, oy = ya - yb;
      dx = (T)dcx + ox;
      dy = (T)dcy + oy;
    }
  }

  // Separation a - b for b in the cell (ox, oy) away from a's cell (|ox|, |oy| <= 1
  // after the periodic wrap, so the minimum-image cell difference is -ox, -oy).
  __device__ static void sep_nb(const Consts<T> &k, int ox, int oy, T xa, T ya, T xb, T yb, T &dx, T &dy) {
    if constexpr (G) {
      sep(k, 0, xa, ya, 0, xb, yb, dx, dy);
    } else {
      T o1 = xa - xb, o2 = ya - yb;
      dx = (T)(-ox) + o1;
      dy = (T)(-oy) + o2;
    }
  }

  // Bilinear stencil origin (i0, j0) and fractions (tx, ty) for s = P - (1/2, 1/2);
  // (cx, cy) is the particle's cell.
  __device__ static void stencil(const Consts<T> &k, int cx, int cy, T x, T y, int &i0, int &j0, T &tx, T &ty) {
    if constexpr (G) {
      T sx = x - (T)0.5, sy = y - (T)0.5;
      T fx = floor(sx), fy = floor(sy);
      tx = sx - fx;
      ty = sy - fy;
      i0 = (int)fx;
      j0 = (int)fy;
    } else {
      if (x >= (T)0.5) {
        i0 = cx;
        tx = x - (T)0.5;
      } else {
        i0 = cx - 1;
        tx = x + (T)0.5;
      }
      if (y >= (T)0.5) {
        j0 = cy;
        ty = y - (T)0.5;
      } else {
        j0 = cy - 1;
        ty = y + (T)0.5;
      }
    }
  }

  // Move by v (P <- P + v), then periodic wrap or wall mirror.  Returns the new
  // cell key, or -1 if the result is not a valid cell (NaN, or a jump across
  // the whole domain).  wy: +1 if a move periodic in y ended at or beyond
  // y = ny (wrapped to the bottom), -1 if it ended below 0, else 0.
  __device__ static int move(const Consts<T> &k, int cx, int cy, T &x, T &y, T vx, T vy, int &wy) {
    wy = 0;
    if constexpr (G) {
      T X = x + vx, Y = y + vy;
      if (k.per_y) wy = Y >= (T)k.ny ? 1 : (Y < (T)0 ? -1 : 0);
      X = k.per_x ? wrap_c(X, (T)k.nx) : mirror_c(X, (T)k.nx);
      Y = k.per_y ? wrap_c(Y, (T)k.ny) : mirror_c(Y, (T)k.ny);
      x = X;
      y = Y;
      T fx = floor(X), fy = floor(Y);
      if (!(fx >= (T)0 && fx < (T)k.nx && fy >= (T)0 && fy < (T)k.ny)) return -1;
      return (int)fy * k.nx + (int)fx;
    } else {
      T ox = x + vx, oy = y + vy;
      renorm(ox, cx);
      renorm(oy, cy);
      if (k.per_y) wy = cy >= k.ny ? 1 : (cy < 0 ? -1 : 0);
      if (!axis(cx, ox, k.nx, k.per_x) || !axis(cy, oy, k.ny, k.per_y)) return -1;
      x = ox;
      y = oy;
      return cy * k.nx + cx;
    }
  }

  __device__ static T wrap_c(T x, T L) {
    if (x >= L) {
      x -= L;
    } else if (x < (T)0) {
      x += L;
      if (x >= L) x = (T)0;
    }
    return x;
  }
  __device__ static T mirror_c(T x, T L) {
    if (x < (T)0) x = -x;
    if (x >= L) x = (T)2 * L - x;
    if (x >= L) x = nextafter(L, (T)0);
    return x;
  }
  // Offset in [0, 1) after adding a displacement; carries into the cell index.
  __device__ static void renorm(T &o, int &c) {
    if (o >= (T)1 || o < (T)0) {
      T fl = floor(o);
      o -= fl;
      c += (int)fl;
      if (o >= (T)1) {
        o = (T)0;
        c += 1;
      }
    }
  }
  // Periodic wrap or wall mirror of a (cell, offset) coordinate.
  __device__ static bool axis(int &c, T &o, int n, int per) {
    if (c >= 0 && c < n) return true;
    if (per) {
      c = ((c % n) + n) % n;
      return true;
    }
    if (c < 0) {  // mirror at 0: -(c + o) = (-c - 1) + (1 - o)
      c = -c - 1;
      o = (T)1 - o;
    } else {  // mirror at n: 2n - (c + o) = (2n - c - 1) + (1 - o)
      c = 2 * n - c - 1;
      o = (T)1 - o;
    }
    if (o >= (T)1) {
      o = (T)0;
      c += 1;
    }
    if (c >= n) {
      c = n - 1;
      o = (T)0.99999994f;
    }
    return c >= 0 && c < n;
  }

  // Global coordinate along x / y as FP64 (exact for both representations).
  __device__ static double gx(const Consts<T> &k, int key, T x) {
    if constexpr (G) return (double)x;
    else return (double)(key - cell_row(k, key) * k.nx) + (double)x;
  }
  __device__ static double gy(const Consts<T> &k, int key, T y) {
    if constexpr (G) return (double)y;
    else return (double)cell_row(k, key) + (double)y;
  }

  __device__ static int walls_key(const Consts<T> &k, int key, T x, T y, T &vx, T &vy) {
    int cx, cy;
    cell_xy(k, key, cx, cy);
    return walls(k, cx, cy, x, y, vx, vy);
  }

  // Particle-wall collisions on non-periodic axes (walls as infinitely heavy
  // particles, Sec. 2.2): within r of a wall and moving into it, v_n -> -e_w v_n.
  // Faces in the order x-, x+, y-, y+.
  __device__ static int walls(const Consts<T> &k, int cx, int cy, T x, T y, T &vx, T &vy) {
    int hits = 0;
    bool lx, rx, ly, ry;
    if constexpr (G) {
      lx = x <= k.r;
      rx = (T)k.nx - x <= k.r;
      ly = y <= k.r;
      ry = (T)k.ny - y <= k.r;
    } else {
      lx = cx == 0 && x <= k.r;
      rx = cx == k.nx - 1 && (T)1 - x <= k.r;
      ly = cy == 0 && y <= k.r;
      ry = cy == k.ny - 1 && (T)1 - y <= k.r;
    }
    if (!k.per_x) {
      if (lx && vx < (T)0) {
        vx = -k.e_pw * vx;
        ++hits;
      }
      if (rx && vx > (T)0) {
        vx = -k.e_pw * vx;
        ++hits;
      }
    }
    if (!k.per_y) {
      if (ly && vy < (T)0) {
        vy = -k.e_pw * vy;
        ++hits;
      }
      if (ry && vy > (T)0) {
        vy = -k.e_pw * vy;
        ++hits;
      }
    }
    return hits;
  }
};

// Neighbour rows: particle u's contacts, sorted by particle index, as 64-bit
// entries (index << 32 | slot).  The first ADJ_IN entries of every row are
// stored densely ([N][ADJ_IN], one 32-byte run per particle); entries
// ADJ_IN .. KMAX-1, which few particles have, in a second array
// ([N][KMAX - ADJ_IN]).
constexpr int ADJ_IN = 4;
struct AdjRow {
  long long *a, *b;
  __device__ long long &operator[](int i) const { return i < ADJ_IN ? a[i] : b[i - ADJ_IN]; }
};
// The dense part of a row held in registers; get() selects an entry without
// indexing (which would put the values in scratch memory).
struct Dense4 {
  long long e0, e1, e2, e3;
  __device__ explicit Dense4(const long long *a) : e0(a[0]), e1(a[1]), e2(a[2]), e3(a[3]) {}
  __device__ long long get(int i) const { return i == 0 ? e0 : (i == 1 ? e1 : (i == 2 ? e2 : e3)); }
};
static_assert(ADJ_IN == 4, "Dense4 holds the dense part of a row");
struct Adj {
  long long *in, *ov;
  __device__ AdjRow row(int u) const {
    return AdjRow{in + (size_t)u * ADJ_IN, ov + (size_t)u * (KMAX - ADJ_IN)};
  }
};

// Generic three-pass scan: SCAN_ITEMS per thread.
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = BLOCK * SCAN_ITEMS;
// Cell-start scan: tiles of SCAN_TILE = 2^shift cells.  The per-tile particle
// counts of the next binning are accumulated while the new cells are counted
// (one atomic per workgroup and tile).
struct TileSums {
  int32_t *tile;
  int ntiles, shift;
  __device__ void add(int t, int v) const { atomicAdd(&tile[t], v); }
};

constexpr int LUT_ROWS_MAX = 64;              // per-count table rows staged in LDS
constexpr int RANK_MOVED = 1 << 30;           // rank flag: the particle arrived from another cell
constexpr int SEG_REG = 4;                    // cell segments up to this length stay in registers
constexpr int CONTACT_REG = 4;                // contacts per particle collected in registers first
constexpr int CONTACT_CH = 4;                 // candidate positions loaded together
constexpr int CONTACT_W = 2;                  // slots each side of a particle loaded before its cell starts
constexpr int CONTACT_W_SMALL = 3;            // the same for grids that fit on the chip at six waves per SIMD
constexpr int RES_ITEMS = 8;                  // particle indices per lane and resolution chunk
// done[] of a particle whose whole cluster the cluster kernel resolved (its
// pairs and its wall pass): the ordered sweep leaves it alone.  A particle of
// a cluster left to the sweep keeps the plain count of its finished pairs.
constexpr int DONE_WHOLE = 1 << 30;
constexpr int RES_CHUNK = BLOCK * RES_ITEMS;  // particle indices per chunk

// Block-wide exclusive scan of one int per thread; total = block sum.
__device__ __forceinline__ int block_excl_scan(int v, int *sh, int &total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int inc = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(inc, o, 64);
    if (lane >= o) inc += u;
  }
  if (lane == 63) sh[wv] = inc;
  __syncthreads();
  int base = 0;
  total = 0;
  for (int w = 0; w < BLOCK / 64; ++w) {
    if (w < wv) base += sh[w];
    total += sh[w];
  }
  __syncthreads();
  return base + inc - v;
}

// Block-wide exclusive scan of one 64-bit integer per thread; total = block sum.
__device__ __forceinline__ long long block_excl_scan_ll(long long v, long long *sh, long long &total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  long long inc = v;
  for (int o = 1; o < 64; o <<= 1) {
    const long long u = __shfl_up(inc, o, 64);
    if (lane >= o) inc += u;
  }
  if (lane == 63) sh[wv] = inc;
  __syncthreads();
  long long base = 0;
  total = 0;
  for (int w = 0; w < BLOCK / 64; ++w) {
    if (w < wv) base += sh[w];
    total += sh[w];
  }
  __syncthreads();
  return base + inc - v;
}

// Block-wide sums of two non-negative counts (each total below 2^31) in one
// pass: packed as a << 32 | b, so one reduction and one pair of barriers
// serve both.  Valid in thread 0.
__device__ __forceinline__ void block_sum2(long long a, long long b, long long *sh, long long &ta, long long &tb) {
  long long v = (a << 32) + b;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  long long t = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < BLOCK / 64; ++w) t += sh[w];
  __syncthreads();
  ta = t >> 32;
  tb = t & 0xffffffffll;
}

// Block-wide sum of a 64-bit integer (BLOCK threads), result valid in thread 0.
__device__ __forceinline__ long long block_sum_ll(long long v, long long *sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  long long t = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < BLOCK / 64; ++w) t += sh[w];
  __syncthreads();
  return t;
}

// ------------------------------------------------------------------ A2 + A3: deposition fused into collide-stream
// One thread per cell.  Reads the cell's particle segment (sorted by cell, then
// particle index) to form n_tot and v_s (Eq. 8), the nine pre-collision
// populations, collides with Eq. 23 (solid term Eq. 7, weights Eqs. 9-11, 20),
// writes rho, the actual gas velocity (Eq. 24 and note), F_p->g (Eq. 25) and
// beta (Eqs. 19, 21, 22), and pushes the post-collision populations to their
// neighbours with the boundary rules (bounce-back, equilibrium inlet,
// zero-gradient outlet).
template <int P>
__device__ __forceinline__ void collide_body(const int bidx, const int gdim,
    const typename Prec<P>::S *__restrict__ fsrc, typename Prec<P>::S *__restrict__ fdst,
    Fields<typename Prec<P>::T> fl, const int32_t *__restrict__ cs, Parts<typename Prec<P>::T> pt,
    const typename Prec<P>::T *__restrict__ lut, const typename Prec<P>::T *__restrict__ inlet,
    Consts<typename Prec<P>::T> k, int32_t *dg_n, typename Prec<P>::T *dg_vsx, typename Prec<P>::T *dg_vsy) {
  using T = typename Prec<P>::T;
  __shared__ T sl[LUT_ROWS_MAX * LUT_W];  // the per-count table
  const int c = bidx * BLOCK + threadIdx.x;
  const bool live = c < k.C;
  const size_t C = (size_t)k.C;
  // the cell's populations and segment bounds are requested before the table
  // is staged, so the two memory round trips overlap
  T f[Q];  // f_i (FP64) or g_i = f_i - w_i
  int a0 = 0, a1 = 0;
  if (live) {
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = load_v<P>(fsrc, i * C + c);
    a0 = cs[c];
    a1 = cs[c + 1];
  }
  for (int i = threadIdx.x; i < min(k.nlut, LUT_ROWS_MAX) * LUT_W; i += BLOCK) sl[i] = lut[i];
  __syncthreads();
  if (!live) return;
  int x, y;
  cell_xy(k, c, x, y);

  // The binning leaves each cell's particles in arrival order: put the
  // segment in ascending particle index (a segment already in order is only
  // read).  Later stages of this step sum over the segment in that order.
  // Up to SEG_REG particles are handled in registers, longer segments by an
  // insertion sort of the records in memory.
  const int n = a1 - a0;
  T sx = (T)0, sy = (T)0;
  if (n <= SEG_REG) {
    int id[SEG_REG];
    T px[SEG_REG], py[SEG_REG], vx[SEG_REG], vy[SEG_REG];
#pragma unroll
    for (int u = 0; u < SEG_REG; ++u)
      if (u < n) {
        id[u] = pt.pid[a0 + u];
        vx[u] = pt.vx[a0 + u];
        vy[u] = pt.vy[a0 + u];
      }
    bool moved = false, unsorted = false;
#pragma unroll
    for (int q = 0; q < SEG_REG - 1; ++q) unsorted |= q + 1 < n && id[q] > id[q + 1];
    if (unsorted) {  // positions are needed only to move records: usually the cell is in order
#pragma unroll
      for (int u = 0; u < SEG_REG; ++u)
        if (u < n) {
          px[u] = pt.px[a0 + u];
          py[u] = pt.py[a0 + u];
        }
    }
    if (unsorted)
#pragma unroll
    for (int pass = 0; pass < SEG_REG - 1; ++pass)
#pragma unroll
      for (int q = 0; q < SEG_REG - 1; ++q)
        if (q + 1 < n && id[q] > id[q + 1]) {
          int ti = id[q];
          id[q] = id[q + 1];
          id[q + 1] = ti;
          T t0 = px[q];
          px[q] = px[q + 1];
          px[q + 1] = t0;
          t0 = py[q];
          py[q] = py[q + 1];
          py[q + 1] = t0;
          t0 = vx[q];
          vx[q] = vx[q + 1];
          vx[q + 1] = t0;
          t0 = vy[q];
          vy[q] = vy[q + 1];
          vy[q + 1] = t0;
          moved = true;
        }
    if (moved) {
#pragma unroll
      for (int u = 0; u < SEG_REG; ++u)
        if (u < n) {
          pt.pid[a0 + u] = id[u];
          pt.px[a0 + u] = px[u];
          pt.py[a0 + u] = py[u];
          pt.vx[a0 + u] = vx[u];
          pt.vy[a0 + u] = vy[u];
        }
    }
    // Eq. 8: n_tot and v_s, summed in ascending particle index.
#pragma unroll
    for (int u = 0; u < SEG_REG; ++u)
      if (u < n) {
        sx += vx[u];
        sy += vy[u];
      }
  } else {
    for (int i = a0 + 1; i < a1; ++i) {
      const int kv = pt.pid[i];
      if (pt.pid[i - 1] <= kv) continue;
      const T x0 = pt.px[i], y0 = pt.py[i], u0 = pt.vx[i], w0 = pt.vy[i];
      int j = i - 1;
      do {
        pt.pid[j + 1] = pt.pid[j];
        pt.px[j + 1] = pt.px[j];
        pt.py[j + 1] = pt.py[j];
        pt.vx[j + 1] = pt.vx[j];
        pt.vy[j + 1] = pt.vy[j];
        --j;
      } while (j >= a0 && pt.pid[j] > kv);
      pt.pid[j + 1] = kv;
      pt.px[j + 1] = x0;
      pt.py[j + 1] = y0;
      pt.vx[j + 1] = u0;
      pt.vy[j + 1] = w0;
    }
    // Eq. 8: n_tot and v_s, summed in ascending particle index.
    for (int s = a0; s < a1; ++s) {
      sx += pt.vx[s];
      sy += pt.vy[s];
    }
  }
  T vsx = (T)0, vsy = (T)0;
  if (n > 0) {
    vsx = dv<P>(sx, (T)n);
    vsy = dv<P>(sy, (T)n);
  }
  const int row = min(n, k.nlut - 1);
  const T *L = row < LUT_ROWS_MAX ? sl + row * LUT_W : lut + (size_t)row * LUT_W;

  T rho = (T)0, rho1 = (T)0, jx = (T)0, jy = (T)0;
  if constexpr (kDev<P>) {
#pragma unroll
    for (int i = 0; i < Q; ++i) rho1 += f[i];
    rho = (T)1.0 + rho1;
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) rho += f[i];
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) jx += (T)cx_of(i) * f[i];
#pragma unroll
  for (int i = 0; i < Q; ++i) jy += (T)cy_of(i) * f[i];
  const T ux = dv<P>(jx, rho), uy = dv<P>(jy, rho);
  T fu[Q], oms[Q], fs[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) fu[i] = feq_v<P>(i, rho, rho1, ux, uy);
  // Eq. 7 (the weights cancel between f_-i and f_i, so the same form holds for deviations)
#pragma unroll
  for (int i = 0; i < Q; ++i) oms[i] = f[opp9(i)] - f[i] + feq_v<P>(i, rho, rho1, vsx, vsy) - fu[opp9(i)];
  const T omg = L[L_OMG];
  T relax = L[L_RELAX];
  if (k.les) {
    // Smagorinsky sub-grid model (Eqs. 12-15): the momentum flux of the
    // non-equilibrium part, Q_ij = sum_k c_ki c_kj (f_k - f_k^eq) (Eq. 13), its
    // norm Q = sqrt(2 Q_ij Q_ij), and tau_t, the positive root of
    // tau_t^2 - tau tau_t - 9 C_s^2 Q / (2 rho) = 0 (Eqs. 12-14; Eq. 15 with
    // Q / rho).  The BGK part relaxes with 1/tau_t and gamma(eps_s, tau_t)
    // (Eq. 23); the solid term keeps gamma(eps_s, tau).  Deviations cancel in
    // f - f^eq, so every storage mode forms the same Q_ij.
    T qxx = (T)0, qyy = (T)0, qxy = (T)0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const T ne = f[i] - fu[i];
      qxx += (T)(cx_of(i) * cx_of(i)) * ne;
      qyy += (T)(cy_of(i) * cy_of(i)) * ne;
      qxy += (T)(cx_of(i) * cy_of(i)) * ne;
    }
    const T q = sq<P>((T)2.0 * (qxx * qxx + qyy * qyy + (T)2.0 * (qxy * qxy)));
    const T tt = (T)0.5 * (k.tau + sq<P>(k.tau * k.tau + dv<P>(k.cs18 * q, rho)));
    const T es2 = L[L_ES2];
    const T gt = dv<P>(es2 * (tt - (T)0.5), ((T)1.0 - es2) + (tt - (T)0.5));
    relax = dv<P>((T)1.0 - gt, tt);
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) fs[i] = f[i] - relax * (f[i] - fu[i]) + omg * oms[i] + k.src[i];
  T ssx = (T)0, ssy = (T)0;
#pragma unroll
  for (int i = 0; i < Q; ++i) ssx += (T)cx_of(i) * oms[i];
#pragma unroll
  for (int i = 0; i < Q; ++i) ssy += (T)cy_of(i) * oms[i];
  const T fpx = omg * ssx, fpy = omg * ssy;
  const T usx = dv<P>(jx + (T)0.5 * fpx + k.halfG[0], rho);
  const T usy = dv<P>(jy + (T)0.5 * fpy + k.halfG[1], rho);
  const T ugx = dv<P>(usx, L[L_UDIV]), ugy = dv<P>(usy, L[L_UDIV]);
  const T ddx = ugx - vsx, ddy = ugy - vsy;
  const T slip = sq<P>(ddx * ddx + ddy * ddy);
  T beta;
  if (L[L_DILUTE] != (T)0) {
    const T re = dv<P>(L[L_BRE] * slip * k.d, k.mu);
    if (re < (T)1000)
      beta = L[L_A] * ((T)1.0 + (T)0.15 * pw<P>(re, (T)0.687));
    else
      beta = dv<P>(L[L_H] * slip * (T)0.44 * L[L_OM], k.d);
  } else {
    beta = L[L_D1] + dv<P>(L[L_D2] * slip, k.d);
  }
  fl.rho[c] = kDev<P> ? rho1 : rho;  // the deviation modes keep rho - 1
  fl.ugx[c] = ugx;
  fl.ugy[c] = ugy;
  fl.beta[c] = beta;
  fl.fpgx[c] = fpx;
  fl.fpgy[c] = fpy;
  fl.es[c] = L[L_ES3];
  if (dg_n) {
    dg_n[c] = n;
    dg_vsx[c] = vsx;
    dg_vsy[c] = vsy;
  }

  // Streaming, push form.  An x wall takes precedence at corners.
  if (x >= 1 && x < k.nx - 1 && y >= 1 && y < k.ny - 1) {  // interior: every neighbour is a lattice node
#pragma unroll
    for (int i = 0; i < Q; ++i) store_v<P>(fdst, i * C + c + cy_of(i) * k.nx + cx_of(i), fs[i]);
    return;
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    int tx = x + cx_of(i), ty = y + cy_of(i);
    if (tx < 0 || tx >= k.nx) {
      if (!k.per_x) {  // halfway bounce-back: returns as the opposite population
        store_v<P>(fdst, opp9(i) * C + c, fs[i]);
        continue;
      }
      tx = wrap_i(tx, k.nx);
    }
    if (ty < 0 || ty >= k.ny) {
      const int face = ty < 0 ? k.bc_ylo : k.bc_yhi;
      if (face == BC_PERIODIC) {
        ty = wrap_i(ty, k.ny);
      } else if (face == BC_WALL) {
        store_v<P>(fdst, opp9(i) * C + c, fs[i]);
        continue;
      } else {
        continue;  // leaves through an inlet or outlet face
      }
    }
    store_v<P>(fdst, i * C + (size_t)ty * k.nx + tx, fs[i]);
  }
  // Populations entering through an inlet or outlet face.
  if ((y == 0 && k.bc_ylo >= BC_INLET) || (y == k.ny - 1 && k.bc_yhi >= BC_INLET)) {
    const int face = y == 0 ? k.bc_ylo : k.bc_yhi;
    const int dir = y == 0 ? 1 : -1;  // c_y of the entering populations
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      if (cy_of(i) != dir) continue;
      if (face == BC_INLET) {
        // f_i(x) = f^eq_i(1, (0, u_in(x))) unless its source lies beyond an x wall
        const int sxn = x - cx_of(i);
        if ((sxn < 0 || sxn >= k.nx) && !k.per_x) continue;
        store_v<P>(fdst, i * C + c, feq_v<P>(i, (T)1.0, (T)0.0, (T)0.0, inlet[x]));
      } else {
        // zero gradient: this boundary node also feeds its own row
        int tx = x + cx_of(i);
        if (tx < 0 || tx >= k.nx) {
          if (!k.per_x) continue;
          tx = wrap_i(tx, k.nx);
        }
        store_v<P>(fdst, i * C + (size_t)y * k.nx + tx, fs[i]);
      }
    }
  }
}
template <int P>
__global__ __launch_bounds__(BLOCK) void k_collide(const typename Prec<P>::S *__restrict__ fsrc,
                                                   typename Prec<P>::S *__restrict__ fdst,
                                                   Fields<typename Prec<P>::T> fl, const int32_t *__restrict__ cs,
                                                   Parts<typename Prec<P>::T> pt,
                                                   const typename Prec<P>::T *__restrict__ lut,
                                                   const typename Prec<P>::T *__restrict__ inlet,
                                                   Consts<typename Prec<P>::T> k, int32_t *dg_n,
                                                   typename Prec<P>::T *dg_vsx, typename Prec<P>::T *dg_vsy) {
  collide_body<P>(xcd_block<XCD_RUN_COLLIDE>(blockIdx.x, gridDim.x), gridDim.x, fsrc, fdst, fl, cs, pt, lut, inlet, k, dg_n, dg_vsx, dg_vsy);
}

// One symplectic Euler step of length h = 1 / n_sub of Eq. 16 for the particle
// in slot s of cell (cx, cy) = c: v <- v + a h, P <- P + v h, then the periodic
// wrap or wall mirror.  Stores the record and returns the new cell (the old
// one, with the domain flag raised, if the result is not a valid cell).
template <int P>
__device__ __forceinline__ int advance_one(const Consts<typename Prec<P>::T> &k, Parts<typename Prec<P>::T> &pt,
                                           int s, int cx, int cy, int c, typename Prec<P>::T x,
                                           typename Prec<P>::T y, typename Prec<P>::T vx, typename Prec<P>::T vy,
                                           typename Prec<P>::T ax, typename Prec<P>::T ay, int32_t *flags) {
  vx = vx + ax * k.h;
  vy = vy + ay * k.h;
  int wy;
  int nk = Pos<P>::move(k, cx, cy, x, y, vx * k.h, vy * k.h, wy);
  if (wy) atomicAdd(k.cross, (unsigned long long)(long long)wy);  // two's complement: -1 subtracts one
  if (nk < 0) {
    atomicOr(&flags[FLAG_DOMAIN], 1);
    nk = c;
  }
  pt.key[s] = nk;
  pt.px[s] = x;
  pt.py[s] = y;
  pt.vx[s] = vx;
  pt.vy[s] = vy;
  return nk;
}

// ------------------------------------------------------------------ A4 + A5: drag and integration, fused with binning
// One thread per cell, looping over its particles (ascending index).  Pass 1
// interpolates u_gas, the solid fraction, beta and grad p at each particle
// (bilinear, Sec. 2.3 after Eq. 26), forms the pre-estimated drag (Eq. 26) and
// the cell sum (Eq. 27).  Pass 2 distributes F_p->g with Eq. 28, integrates
// Eq. 16 (symplectic Euler), moves, wraps or mirrors, and counts the particle
// into its new cell for the next binning.
// Node fields a workgroup's particles interpolate from, staged in LDS: the
// workgroup covers a TX x TY tile of cells (TX TY = BLOCK), and its particles'
// bilinear stencils reach one node beyond it on every side.  Each slot holds
// the value at the wrapped (periodic) or clamped (wall) node, and the node's
// pressure gradient is formed from the node's own neighbours as in the global
// field.  Three tile shapes are built, 32 x 8, 64 x 4 and 128 x 2 (the
// tuning's drag_tile 0, 1, 2); every result is the same bit for bit, only the
// halo (the staged nodes per cell) and the length of each row's contiguous run
// of particle slots differ.
constexpr int DRAG_TILES = 3;
__host__ __device__ constexpr int drag_tile_w(int t) { return t == 1 ? 64 : (t == 2 ? 128 : 32); }
template <int TX> struct TileDims {
  static_assert(BLOCK % TX == 0, "a tile holds BLOCK cells");
  static constexpr int TY = BLOCK / TX, SX = TX + 2, SY = TY + 2, SN = SX * SY;
};
constexpr int HIST_MAX = 32;

// Eq. 28's denominator as used: the cell's sum S of pre-drags (Eq. 27), or
// zero, so that F_p->g is split equally as for an exactly zero sum, where the
// regularised mode finds the pre-drags cancelling: sum |F_pre| above
// DRAG_CANCEL_MAX |S|, where the ratio of Eq. 28 would turn a small gas force
// into large opposite kicks.
constexpr float DRAG_CANCEL_MAX = 100.0f;
template <class T> __device__ __forceinline__ T drag_den(const Consts<T> &k, T S, T A) {
  return (k.drag_reg && A > (T)DRAG_CANCEL_MAX * fabs(S)) ? (T)0 : S;
}

template <int P, int TX> struct DragTile {
  using T = typename Prec<P>::T;
  static constexpr int DTX = TX, DTY = TileDims<TX>::TY, DSX = TileDims<TX>::SX, DSN = TileDims<TX>::SN;
  T ux[DSN], uy[DSN], es[DSN], beta[DSN], gpx[DSN], gpy[DSN];

  // A thread's share of the tile (slots threadIdx.x + r BLOCK), fetched into
  // registers first and stored into the tile after the workgroup has decided
  // to stay, so the fetch overlaps the first round trip of the kernel.
  static constexpr int R = (DSN + BLOCK - 1) / BLOCK;
  struct Regs {
    T ux[R], uy[R], beta[R], es[R], re[R], rw[R], rn[R], rs[R];
  };
  __device__ static void fetch(const Consts<T> &k, const Fields<T> &fl, int tx0, int ty0, Regs &g) {
    // the tile and its two-node border inside the lattice: no wrapping or clamping
    const bool inner = tx0 >= 2 && tx0 + DTX + 2 <= k.nx && ty0 >= 2 && ty0 + DTY + 2 <= k.ny;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int q = threadIdx.x + r * BLOCK;
      if (q < DSN) {
        const int x = tx0 - 1 + q % DSX, y = ty0 - 1 + q / DSX;
        int c, ie, iw, jn, js;
        if (inner) {
          c = y * k.nx + x;
          ie = c + 1;
          iw = c - 1;
          jn = c + k.nx;
          js = c - k.nx;
        } else {
          const int i = node_idx(x, k.nx, k.per_x), j = node_idx(y, k.ny, k.gas_per_y);
          const int row = j * k.nx;
          c = row + i;
          // the boundary value serves as the ghost beyond a wall
          ie = row + node_idx(i + 1, k.nx, k.per_x);
          iw = row + node_idx(i - 1, k.nx, k.per_x);
          jn = node_idx(j + 1, k.ny, k.gas_per_y) * k.nx + i;
          js = node_idx(j - 1, k.ny, k.gas_per_y) * k.nx + i;
        }
        g.ux[r] = ldu(fl.ugx, c);
        g.uy[r] = ldu(fl.ugy, c);
        g.beta[r] = ldu(fl.beta, c);
        g.es[r] = ldu(fl.es, c);
        // central differences of p = rho / 3
        g.re[r] = ldu(fl.rho, ie);
        g.rw[r] = ldu(fl.rho, iw);
        g.rn[r] = ldu(fl.rho, jn);
        g.rs[r] = ldu(fl.rho, js);
      }
    }
  }
  __device__ void store(const Regs &g) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int q = threadIdx.x + r * BLOCK;
      if (q < DSN) {
        ux[q] = g.ux[r];
        uy[q] = g.uy[r];
        beta[q] = g.beta[r];
        es[q] = g.es[r];
        gpx[q] = (dv<P>(g.re[r], (T)3.0) - dv<P>(g.rw[r], (T)3.0)) * (T)0.5;
        gpy[q] = (dv<P>(g.rn[r], (T)3.0) - dv<P>(g.rs[r], (T)3.0)) * (T)0.5;
      }
    }
  }
};

// Interpolated gas quantities at one particle (bilinear, Sec. 2.3 after Eq. 26).
template <int P> struct Interp {
  using T = typename Prec<P>::T;
  T ux, uy, es, beta, gpx, gpy;

  template <int TX>
  __device__ void at(const Consts<T> &k, const DragTile<P, TX> &D, int tx0, int ty0, int cx, int cy, T x, T y) {
    constexpr int DSX = TileDims<TX>::SX;
    int i0, j0;
    T tx, ty;
    Pos<P>::stencil(k, cx, cy, x, y, i0, j0, tx, ty);
    const int q = (j0 - ty0 + 1) * DSX + (i0 - tx0 + 1);
    const int qq[4] = {q, q + 1, q + DSX, q + DSX + 1};
    const T w[4] = {((T)1.0 - tx) * ((T)1.0 - ty), tx * ((T)1.0 - ty), ((T)1.0 - tx) * ty, tx * ty};
    ux = w[0] * D.ux[qq[0]] + w[1] * D.ux[qq[1]] + w[2] * D.ux[qq[2]] + w[3] * D.ux[qq[3]];
    uy = w[0] * D.uy[qq[0]] + w[1] * D.uy[qq[1]] + w[2] * D.uy[qq[2]] + w[3] * D.uy[qq[3]];
    es = w[0] * D.es[qq[0]] + w[1] * D.es[qq[1]] + w[2] * D.es[qq[2]] + w[3] * D.es[qq[3]];
    beta = w[0] * D.beta[qq[0]] + w[1] * D.beta[qq[1]] + w[2] * D.beta[qq[2]] + w[3] * D.beta[qq[3]];
    gpx = w[0] * D.gpx[qq[0]] + w[1] * D.gpx[qq[1]] + w[2] * D.gpx[qq[2]] + w[3] * D.gpx[qq[3]];
    gpy = w[0] * D.gpy[qq[0]] + w[1] * D.gpy[qq[1]] + w[2] * D.gpy[qq[2]] + w[3] * D.gpy[qq[3]];
  }
};

// Workgroup = one DTX x DTY tile of cells, one thread per cell (its particles
// in registers up to SEG_REG of them, in two passes over memory beyond).
template <int P, int DTX>
__device__ __forceinline__ void drag_body_cells(const int bidx, const int gdim, Parts<typename Prec<P>::T> pt,
    Fields<typename Prec<P>::T> fl, const int32_t *__restrict__ cs, const typename Prec<P>::T *__restrict__ lut,
    Consts<typename Prec<P>::T> k, int32_t *__restrict__ count, int32_t *__restrict__ rank, int32_t *flags,
    typename Prec<P>::T *dg_fdx, typename Prec<P>::T *dg_fdy, long long *zero_part, TileSums ts,
    int32_t *__restrict__ stay) {
  using T = typename Prec<P>::T;
  __shared__ long long sh[BLOCK / 64];
  __shared__ int hist[HIST_MAX];
  constexpr int DTY = TileDims<DTX>::TY;
  __shared__ DragTile<P, DTX> D;
  const int ntx = (k.nx + DTX - 1) / DTX;
  const int tx0 = (bidx % ntx) * DTX, ty0 = (bidx / ntx) * DTY;
  const int cx = tx0 + (int)threadIdx.x % DTX, cy = ty0 + (int)threadIdx.x / DTX;
  const int c = cy * k.nx + cx;
  const bool inside = cx < k.nx && cy < k.ny;
  const int a0 = inside ? cs[c] : 0, a1 = inside ? cs[c + 1] : 0;
  const int n = a1 - a0;
  typename DragTile<P, DTX>::Regs tile_regs;
  DragTile<P, DTX>::fetch(k, fl, tx0, ty0, tile_regs);
  // a tile without particles has nothing to do
  if (!__syncthreads_or(n > 0)) {
    if (inside) stay[c] = 0;
    if (zero_part && threadIdx.x == 0) zero_part[bidx] = 0;
    return;
  }
  // this thread's particles (short segments), loaded while the tile is staged
  T px[SEG_REG], py[SEG_REG], pvx[SEG_REG], pvy[SEG_REG];
#pragma unroll
  for (int u = 0; u < SEG_REG; ++u)
    if (u < n) {
      px[u] = pt.px[a0 + u];
      py[u] = pt.py[a0 + u];
      pvx[u] = pt.vx[a0 + u];
      pvy[u] = pt.vy[a0 + u];
    }
  D.store(tile_regs);
  // scan tiles the new cells of this tile's particles can fall in (one cell
  // move at most, periodic jumps go straight to the global counters)
  const int klo = max(0, (ty0 - 1) * k.nx + tx0 - 1);
  const int khi = min(k.C - 1, (ty0 + DTY) * k.nx + tx0 + DTX);
  const int tlo = klo >> ts.shift, nh = (khi >> ts.shift) - tlo + 1;
  if (threadIdx.x < HIST_MAX) hist[threadIdx.x] = 0;
  __syncthreads();
  long long nzero = 0;
  int nstay = 0;
  if (inside) {
    if (n > 0) {
      const T fgx = fl.fpgx[c], fgy = fl.fpgy[c];
      // Eq. 28 for one particle, then Eq. 16: v <- v + g_eff + (F_d + s V_p grad p) / m,
      // P <- P + v, and the particle's new cell.
      auto finish = [&](int s, T prx, T pry, T gpx, T gpy, T Sx, T Sy, T x, T y, T vx, T vy) -> int {
        T fdx, fdy;
        if (Sx == (T)0)
          fdx = dv<P>(-fgx, (T)n);
        else if (k.drag_abs)
          fdx = dv<P>(fabs(fgx), fabs(Sx)) * prx;
        else
          fdx = dv<P>(-fgx * prx, Sx);
        if (Sy == (T)0)
          fdy = dv<P>(-fgy, (T)n);
        else if (k.drag_abs)
          fdy = dv<P>(fabs(fgy), fabs(Sy)) * pry;
        else
          fdy = dv<P>(-fgy * pry, Sy);
        const T ax = k.geff[0] + dv<P>(fdx + k.fp * gpx, k.m);
        const T ay = k.geff[1] + dv<P>(fdy + k.fp * gpy, k.m);
        if (dg_fdx || k.acx) {
          const int id = pt.pid[s];
          if (dg_fdx) {
            dg_fdx[id] = fdx;
            dg_fdy[id] = fdy;
          }
          if (k.acx) {  // held for the later sub-steps, by particle index
            k.acx[id] = ax;
            k.acy[id] = ay;
          }
        }
        return advance_one<P>(k, pt, s, cx, cy, c, x, y, vx, vy, ax, ay, flags);
      };
      // A particle that stays in its cell takes the next rank among the cell's
      // stayers (in segment order); one that moves counts atomically among
      // the arrivals of its new cell, which come after that cell's stayers.
      auto count_new = [&](int s, int nk) {
        if (nk == c) rank[s] = nstay++;
        else rank[s] = atomicAdd(&count[nk], 1) | RANK_MOVED;
        const int dt = (nk >> ts.shift) - tlo;
        if (nh <= HIST_MAX && dt >= 0 && dt < nh)
          atomicAdd(&hist[dt], 1);
        else
          ts.add(nk >> ts.shift, 1);
      };
      if (n <= SEG_REG) {  // short segment: particle data and pre-drags in registers
        T *x = px, *y = py, *vx = pvx, *vy = pvy;
        T prx[SEG_REG], pry[SEG_REG], gpx[SEG_REG], gpy[SEG_REG];
        int nk[SEG_REG];
        T Sx = (T)0, Sy = (T)0;
#pragma unroll
        for (int u = 0; u < SEG_REG; ++u)
          if (u < n) {
            Interp<P> I;
            I.at(k, D, tx0, ty0, cx, cy, x[u], y[u]);
            prx[u] = dv<P>(k.vp * I.beta, I.es) * (I.ux - vx[u]);
            pry[u] = dv<P>(k.vp * I.beta, I.es) * (I.uy - vy[u]);
            gpx[u] = I.gpx;
            gpy[u] = I.gpy;
            Sx += prx[u];
            Sy += pry[u];
          }
        if (k.drag_reg) {  // the sums of |F_pre|, in the same order, after the interpolations
          T Ax = (T)0, Ay = (T)0;
#pragma unroll
          for (int u = 0; u < SEG_REG; ++u)
            if (u < n) {
              Ax += fabs(prx[u]);
              Ay += fabs(pry[u]);
            }
          Sx = drag_den(k, Sx, Ax);
          Sy = drag_den(k, Sy, Ay);
        }
        nzero = (Sx == (T)0) + (Sy == (T)0);
#pragma unroll
        for (int u = 0; u < SEG_REG; ++u)
          if (u < n) nk[u] = finish(a0 + u, prx[u], pry[u], gpx[u], gpy[u], Sx, Sy, x[u], y[u], vx[u], vy[u]);
#pragma unroll
        for (int u = 0; u < SEG_REG; ++u)
          if (u < n) count_new(a0 + u, nk[u]);
      } else {
        T Sx = (T)0, Sy = (T)0, Ax = (T)0, Ay = (T)0;
        for (int s = a0; s < a1; ++s) {
          Interp<P> I;
          I.at(k, D, tx0, ty0, cx, cy, pt.px[s], pt.py[s]);
          const T qx = dv<P>(k.vp * I.beta, I.es) * (I.ux - pt.vx[s]);
          const T qy = dv<P>(k.vp * I.beta, I.es) * (I.uy - pt.vy[s]);
          Sx += qx;
          Sy += qy;
          Ax += fabs(qx);
          Ay += fabs(qy);
        }
        Sx = drag_den(k, Sx, Ax);
        Sy = drag_den(k, Sy, Ay);
        nzero = (Sx == (T)0) + (Sy == (T)0);
        for (int s = a0; s < a1; ++s) {
          Interp<P> I;
          const T x = pt.px[s], y = pt.py[s], vx = pt.vx[s], vy = pt.vy[s];
          I.at(k, D, tx0, ty0, cx, cy, x, y);
          const T prx = dv<P>(k.vp * I.beta, I.es) * (I.ux - vx);
          const T pry = dv<P>(k.vp * I.beta, I.es) * (I.uy - vy);
          count_new(s, finish(s, prx, pry, I.gpx, I.gpy, Sx, Sy, x, y, vx, vy));
        }
      }
    }
    stay[c] = nstay;
  }
  __syncthreads();
  if ((int)threadIdx.x < min(nh, HIST_MAX)) {
    const int h = hist[threadIdx.x];
    if (h) ts.add(tlo + (int)threadIdx.x, h);
  }
  if (zero_part) {
    const long long t = block_sum_ll(nzero, sh);
    if (threadIdx.x == 0) zero_part[bidx] = t;
  }
}
// Workgroup = one DTX x DTY tile of cells.  One thread per cell stages the
// tile; the particles of the tile are then dealt out flat, particle k of the
// tile (in cell order) to thread k mod BLOCK, so that every thread carries one
// to DR_PT particles whatever the spread of the per-cell counts.  Eq. 27's
// cell sums are taken by the cell's own thread from LDS in segment order, so
// every result equals the one-thread-per-cell evaluation bit for bit.  A tile
// holding more than DR_PT BLOCK particles runs one thread per cell instead.
constexpr int DR_PT = 3, DR_CAP = DR_PT * BLOCK;

template <int P, int DTX>
__device__ __forceinline__ void drag_body_flat(const int bidx, const int gdim, Parts<typename Prec<P>::T> pt,
    Fields<typename Prec<P>::T> fl, const int32_t *__restrict__ cs, const typename Prec<P>::T *__restrict__ lut,
    Consts<typename Prec<P>::T> k, int32_t *__restrict__ count, int32_t *__restrict__ rank, int32_t *flags,
    typename Prec<P>::T *dg_fdx, typename Prec<P>::T *dg_fdy, long long *zero_part, TileSums ts,
    int32_t *__restrict__ stay) {
  using T = typename Prec<P>::T;
  __shared__ long long sh[BLOCK / 64];
  __shared__ int shi[BLOCK / 64];
  __shared__ int hist[HIST_MAX];
  constexpr int DTY = TileDims<DTX>::TY;
  __shared__ DragTile<P, DTX> D;
  __shared__ int f_off[BLOCK + 1];   // first flat index of each cell's particles
  __shared__ int f_base[BLOCK];      // slot of flat index j of cell i: f_base[i] + j
  __shared__ short f_cell[DR_CAP];   // cell of each flat index
  __shared__ T f_px[DR_CAP], f_py[DR_CAP];  // pre-drags, then each cell's sums at its first index
  __shared__ unsigned char f_stays[DR_CAP];
  const int ntx = (k.nx + DTX - 1) / DTX;
  const int tx0 = (bidx % ntx) * DTX, ty0 = (bidx / ntx) * DTY;
  const int cx = tx0 + (int)threadIdx.x % DTX, cy = ty0 + (int)threadIdx.x / DTX;
  const int c = cy * k.nx + cx;
  const bool inside = cx < k.nx && cy < k.ny;
  const int a0 = inside ? cs[c] : 0, a1 = inside ? cs[c + 1] : 0;
  const int n = a1 - a0;
  typename DragTile<P, DTX>::Regs tile_regs;
  DragTile<P, DTX>::fetch(k, fl, tx0, ty0, tile_regs);
  // a tile without particles has nothing to do
  if (!__syncthreads_or(n > 0)) {
    if (inside) stay[c] = 0;
    if (zero_part && threadIdx.x == 0) zero_part[bidx] = 0;
    return;
  }
  D.store(tile_regs);
  // scan tiles the new cells of this tile's particles can fall in (one cell
  // move at most, periodic jumps go straight to the global counters)
  const int klo = max(0, (ty0 - 1) * k.nx + tx0 - 1);
  const int khi = min(k.C - 1, (ty0 + DTY) * k.nx + tx0 + DTX);
  const int tlo = klo >> ts.shift, nh = (khi >> ts.shift) - tlo + 1;
  if (threadIdx.x < HIST_MAX) hist[threadIdx.x] = 0;
  long long nzero = 0;
  // Eq. 28 for one particle of cell (pcx, pcy) = pc holding np particles, then
  // Eq. 16: v <- v + g_eff + (F_d + s V_p grad p) / m, P <- P + v, and the
  // particle's new cell.
  auto finish = [&](int s, int pcx, int pcy, int pc, int np, T fgx, T fgy, T prx, T pry, T gpx, T gpy, T Sx, T Sy,
                    T x, T y, T vx, T vy) -> int {
    T fdx, fdy;
    if (Sx == (T)0)
      fdx = dv<P>(-fgx, (T)np);
    else if (k.drag_abs)
      fdx = dv<P>(fabs(fgx), fabs(Sx)) * prx;
    else
      fdx = dv<P>(-fgx * prx, Sx);
    if (Sy == (T)0)
      fdy = dv<P>(-fgy, (T)np);
    else if (k.drag_abs)
      fdy = dv<P>(fabs(fgy), fabs(Sy)) * pry;
    else
      fdy = dv<P>(-fgy * pry, Sy);
    const T ax = k.geff[0] + dv<P>(fdx + k.fp * gpx, k.m);
    const T ay = k.geff[1] + dv<P>(fdy + k.fp * gpy, k.m);
    if (dg_fdx || k.acx) {
      const int id = pt.pid[s];
      if (dg_fdx) {
        dg_fdx[id] = fdx;
        dg_fdy[id] = fdy;
      }
      if (k.acx) {  // held for the later sub-steps, by particle index
        k.acx[id] = ax;
        k.acy[id] = ay;
      }
    }
    return advance_one<P>(k, pt, s, pcx, pcy, pc, x, y, vx, vy, ax, ay, flags);
  };
  // The new cell's count: a particle that stays takes the given rank among its
  // cell's stayers (segment order); one that moves counts atomically among the
  // arrivals of its new cell, which come after that cell's stayers.
  auto count_new = [&](int s, int nk, bool stays, int stay_rank) {
    if (stays) rank[s] = stay_rank;
    else rank[s] = atomicAdd(&count[nk], 1) | RANK_MOVED;
    const int dt = (nk >> ts.shift) - tlo;
    if (nh <= HIST_MAX && dt >= 0 && dt < nh)
      atomicAdd(&hist[dt], 1);
    else
      ts.add(nk >> ts.shift, 1);
  };
  int ptot;
  const int off = block_excl_scan(n, shi, ptot);  // uniform ptot; its barriers order the tile and hist
  if (ptot <= DR_CAP) {
    // ---- flat: particle k of the tile to thread k mod BLOCK
    f_off[threadIdx.x] = off;
    if (threadIdx.x == 0) f_off[BLOCK] = ptot;
    f_base[threadIdx.x] = a0 - off;
    for (int u = 0; u < n; ++u) f_cell[off + u] = (short)threadIdx.x;
    __syncthreads();
    // pre-drags (Eq. 26); the records are read again after the cell sums
    int pcl[DR_PT];
    T prx[DR_PT], pry[DR_PT], gpx[DR_PT], gpy[DR_PT];
#pragma unroll
    for (int j = 0; j < DR_PT; ++j) {
      const int q = (int)threadIdx.x + j * BLOCK;
      if (q < ptot) {
        const int cl = f_cell[q];
        const int s = f_base[cl] + q;
        pcl[j] = cl;
        const T vx = ldu(pt.vx, s), vy = ldu(pt.vy, s);
        Interp<P> I;
        I.at(k, D, tx0, ty0, tx0 + cl % DTX, ty0 + cl / DTX, ldu(pt.px, s), ldu(pt.py, s));
        prx[j] = dv<P>(k.vp * I.beta, I.es) * (I.ux - vx);
        pry[j] = dv<P>(k.vp * I.beta, I.es) * (I.uy - vy);
        gpx[j] = I.gpx;
        gpy[j] = I.gpy;
        f_px[q] = prx[j];
        f_py[q] = pry[j];
      }
    }
    __syncthreads();
    // Eq. 27: the cell's sums in segment order, left at its first flat index
    if (n > 0) {
      T Sx = (T)0, Sy = (T)0, Ax = (T)0, Ay = (T)0;
      for (int u = 0; u < n; ++u) {
        Sx += f_px[off + u];
        Sy += f_py[off + u];
        Ax += fabs(f_px[off + u]);
        Ay += fabs(f_py[off + u]);
      }
      Sx = drag_den(k, Sx, Ax);
      Sy = drag_den(k, Sy, Ay);
      nzero = (Sx == (T)0) + (Sy == (T)0);
      f_px[off] = Sx;
      f_py[off] = Sy;
    }
    __syncthreads();
    int nk[DR_PT];
#pragma unroll
    for (int j = 0; j < DR_PT; ++j) {
      const int q = (int)threadIdx.x + j * BLOCK;
      if (q < ptot) {
        const int cl = pcl[j], o = f_off[cl], s = f_base[cl] + q;
        const int pcx = tx0 + cl % DTX, pcy = ty0 + cl / DTX, pc = pcy * k.nx + pcx;
        nk[j] = finish(s, pcx, pcy, pc, f_off[cl + 1] - o, ldu(fl.fpgx, pc), ldu(fl.fpgy, pc), prx[j], pry[j],
                       gpx[j], gpy[j], f_px[o], f_py[o], ldu(pt.px, s), ldu(pt.py, s), ldu(pt.vx, s), ldu(pt.vy, s));
        f_stays[q] = nk[j] == pc;
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < DR_PT; ++j) {
      const int q = (int)threadIdx.x + j * BLOCK;
      if (q < ptot) {
        const bool st = f_stays[q];
        int r = 0;
        if (st)
          for (int t = f_off[pcl[j]]; t < q; ++t) r += f_stays[t];
        count_new(f_base[pcl[j]] + q, nk[j], st, r);
      }
    }
    if (inside) {
      int ns = 0;
      for (int u = 0; u < n; ++u) ns += f_stays[off + u];
      stay[c] = ns;
    }
  } else {
    // ---- one thread per cell (a tile denser than the flat capacity): two
    // passes over the cell's segment, the sums first
    int nstay = 0;
    if (inside) {
      if (n > 0) {
        const T fgx = fl.fpgx[c], fgy = fl.fpgy[c];
        T Sx = (T)0, Sy = (T)0, Ax = (T)0, Ay = (T)0;
        for (int s = a0; s < a1; ++s) {
          Interp<P> I;
          I.at(k, D, tx0, ty0, cx, cy, pt.px[s], pt.py[s]);
          const T qx = dv<P>(k.vp * I.beta, I.es) * (I.ux - pt.vx[s]);
          const T qy = dv<P>(k.vp * I.beta, I.es) * (I.uy - pt.vy[s]);
          Sx += qx;
          Sy += qy;
          Ax += fabs(qx);
          Ay += fabs(qy);
        }
        Sx = drag_den(k, Sx, Ax);
        Sy = drag_den(k, Sy, Ay);
        nzero = (Sx == (T)0) + (Sy == (T)0);
        for (int s = a0; s < a1; ++s) {
          Interp<P> I;
          const T x = pt.px[s], y = pt.py[s], vx = pt.vx[s], vy = pt.vy[s];
          I.at(k, D, tx0, ty0, cx, cy, x, y);
          const T prx = dv<P>(k.vp * I.beta, I.es) * (I.ux - vx);
          const T pry = dv<P>(k.vp * I.beta, I.es) * (I.uy - vy);
          const int nk = finish(s, cx, cy, c, n, fgx, fgy, prx, pry, I.gpx, I.gpy, Sx, Sy, x, y, vx, vy);
          const bool st = nk == c;
          count_new(s, nk, st, nstay);
          nstay += st;
        }
      }
      stay[c] = nstay;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < min(nh, HIST_MAX)) {
    const int h = hist[threadIdx.x];
    if (h) ts.add(tlo + (int)threadIdx.x, h);
  }
  if (zero_part) {
    const long long t = block_sum_ll(nzero, sh);
    if (threadIdx.x == 0) zero_part[bidx] = t;
  }
}
// Two forms: one thread per cell, for grids that fit on the chip in one round
// (the step is then one chain of round trips, and the flat form's extra
// barriers lengthen it); the flat form for larger grids, where the even
// per-thread work pays: 22 % faster on a 16 M-particle bed, 16 % on a batch of
// 64 uneven beds.
template <int P, int TX>
__global__ __launch_bounds__(BLOCK) LBDPS_WAVES8 void k_drag(Parts<typename Prec<P>::T> pt,
                                                             Fields<typename Prec<P>::T> fl,
                                                             const int32_t *__restrict__ cs,
                                                             const typename Prec<P>::T *__restrict__ lut,
                                                             Consts<typename Prec<P>::T> k,
                                                             int32_t *__restrict__ count, int32_t *__restrict__ rank,
                                                             int32_t *flags, typename Prec<P>::T *dg_fdx,
                                                             typename Prec<P>::T *dg_fdy, long long *zero_part,
                                                             TileSums ts, int32_t *__restrict__ stay) {
  drag_body_cells<P, TX>(xcd_block<XCD_RUN_DRAG>(blockIdx.x, gridDim.x), gridDim.x, pt, fl, cs, lut, k, count, rank,
                         flags, dg_fdx, dg_fdy, zero_part, ts, stay);
}
template <int P, int TX>
__global__ __launch_bounds__(BLOCK) LBDPS_WAVES6 void k_drag_flat(Parts<typename Prec<P>::T> pt, Fields<typename Prec<P>::T> fl,
                                                     const int32_t *__restrict__ cs,
                                                     const typename Prec<P>::T *__restrict__ lut,
                                                     Consts<typename Prec<P>::T> k, int32_t *__restrict__ count,
                                                     int32_t *__restrict__ rank, int32_t *flags,
                                                     typename Prec<P>::T *dg_fdx, typename Prec<P>::T *dg_fdy,
                                                     long long *zero_part, TileSums ts,
                                                     int32_t *__restrict__ stay) {
  drag_body_flat<P, TX>(xcd_block<XCD_RUN_DRAG>(blockIdx.x, gridDim.x), gridDim.x, pt, fl, cs, lut, k, count, rank,
                        flags, dg_fdx, dg_fdy, zero_part, ts, stay);
}

// Sub-steps after the first of a lattice step (n_sub > 1): one thread per
// cell advances the cell's particles by h under the accelerations the drag
// kernel held for their indices, and counts each into its new cell as the
// drag kernel does: a particle that stays takes the next rank among its cell's
// stayers (segment order), one that moves counts atomically among the
// arrivals of its new cell.  A workgroup covers BLOCK consecutive cells; the
// per-tile counts go through a workgroup histogram over the tiles its
// particles can reach in one cell move (periodic jumps go to the global sums).
template <int P>
__device__ __forceinline__ void advance_body(const int bidx, const int gdim, Parts<typename Prec<P>::T> pt,
    Consts<typename Prec<P>::T> k, const int32_t *__restrict__ cs, int32_t *__restrict__ count,
    int32_t *__restrict__ rank, int32_t *__restrict__ stay, int32_t *flags, TileSums ts) {
  using T = typename Prec<P>::T;
  __shared__ int hist[HIST_MAX];
  const int c0 = bidx * BLOCK, c = c0 + (int)threadIdx.x;
  const int tlo = max(0, c0 - k.nx - 1) >> ts.shift;
  const int thi = min(k.C - 1, c0 + BLOCK + k.nx) >> ts.shift;
  const int nh = thi - tlo + 1;
  if (threadIdx.x < HIST_MAX) hist[threadIdx.x] = 0;
  __syncthreads();
  if (c < k.C) {
    const int a0 = cs[c], a1 = cs[c + 1], n = a1 - a0;
    int cx, cy;
    cell_xy(k, c, cx, cy);
    int nstay = 0;
    auto count_new = [&](int s, int nk) {
      if (nk == c) rank[s] = nstay++;
      else rank[s] = atomicAdd(&count[nk], 1) | RANK_MOVED;
      const int dt = (nk >> ts.shift) - tlo;
      if (nh <= HIST_MAX && dt >= 0 && dt < nh)
        atomicAdd(&hist[dt], 1);
      else
        ts.add(nk >> ts.shift, 1);
    };
    if (n <= SEG_REG) {  // short segment: every record loaded before any is advanced
      int id[SEG_REG];
      T x[SEG_REG], y[SEG_REG], vx[SEG_REG], vy[SEG_REG];
#pragma unroll
      for (int u = 0; u < SEG_REG; ++u)
        if (u < n) {
          id[u] = pt.pid[a0 + u];
          x[u] = pt.px[a0 + u];
          y[u] = pt.py[a0 + u];
          vx[u] = pt.vx[a0 + u];
          vy[u] = pt.vy[a0 + u];
        }
#pragma unroll
      for (int u = 0; u < SEG_REG; ++u)
        if (u < n)
          count_new(a0 + u, advance_one<P>(k, pt, a0 + u, cx, cy, c, x[u], y[u], vx[u], vy[u], k.acx[id[u]],
                                           k.acy[id[u]], flags));
    } else {
      for (int s = a0; s < a1; ++s) {
        const int id = pt.pid[s];
        count_new(s, advance_one<P>(k, pt, s, cx, cy, c, pt.px[s], pt.py[s], pt.vx[s], pt.vy[s], k.acx[id],
                                    k.acy[id], flags));
      }
    }
    stay[c] = nstay;
  }
  __syncthreads();
  if ((int)threadIdx.x < min(nh, HIST_MAX)) {
    const int h = hist[threadIdx.x];
    if (h) ts.add(tlo + (int)threadIdx.x, h);
  }
}
template <int P>
__global__ __launch_bounds__(BLOCK) void k_advance(Parts<typename Prec<P>::T> pt, Consts<typename Prec<P>::T> k,
                                                   const int32_t *__restrict__ cs, int32_t *__restrict__ count,
                                                   int32_t *__restrict__ rank, int32_t *__restrict__ stay,
                                                   int32_t *flags, TileSums ts) {
  advance_body<P>(blockIdx.x, gridDim.x, pt, k, cs, count, rank, stay, flags, ts);
}

// ------------------------------------------------------------------ A1: binning (counting sort by cell)
// Count particles per cell (slot within the cell from the atomic counter).
__global__ __launch_bounds__(BLOCK) void k_bin(const int32_t *__restrict__ key, int n, int32_t *__restrict__ count,
                                               int32_t *__restrict__ rank) {
  const int s = blockIdx.x * BLOCK + threadIdx.x;
  if (s < n) rank[s] = atomicAdd(&count[key[s]], 1) | RANK_MOVED;
}

// Move every particle record to its slot cell_start[key] + rank in the other
// storage and record the slot of each particle index.  Clears the tile sums
// for the next binning.
template <class T>
__device__ __forceinline__ void scatter_body(const int bidx, const int gdim, Parts<T> src, Parts<T> dst,
    const int32_t *__restrict__ rank, const int32_t *__restrict__ cs, int n, int32_t *__restrict__ slot, TileSums ts,
    const int32_t *__restrict__ stay) {
  const int s = bidx * BLOCK + threadIdx.x;
  for (int i = s; i < ts.ntiles; i += gdim * BLOCK) ts.tile[i] = 0;
  if (s >= n) return;
  const int key = src.key[s];
  const int r = rank[s];
  const int d = cs[key] + ((r & RANK_MOVED) ? stay[key] + (r & ~RANK_MOVED) : r);
  const int id = src.pid[s];
  dst.key[d] = key;
  dst.pid[d] = id;
  dst.px[d] = src.px[s];
  dst.py[d] = src.py[s];
  dst.vx[d] = src.vx[s];
  dst.vy[d] = src.vy[s];
  slot[id] = d;
}
template <class T>
__global__ __launch_bounds__(BLOCK) void k_scatter(Parts<T> src, Parts<T> dst, const int32_t *__restrict__ rank,
                                                   const int32_t *__restrict__ cs, int n, int32_t *__restrict__ slot,
                                                   TileSums ts, const int32_t *__restrict__ stay) {
  scatter_body<T>(xcd_block<XCD_RUN_SCATTER>(blockIdx.x, gridDim.x), gridDim.x, src, dst, rank, cs, n, slot, ts, stay);
}

// ------------------------------------------------------------------ A6: contact detection
// One thread per particle slot.  Candidates come from the 3x3 cells around the
// particle (d < 1 cell), narrowed to the columns and rows that come within d
// of it; a contact is a centre distance <= d (Sec. 2.2), with the periodic
// minimum image.  Away from a periodic seam the cells of a neighbour row are
// one contiguous slot range, and a candidate's column offset follows from the
// cell starts.  Each particle keeps its full neighbour list
// sorted by particle index, as 64-bit entries (index << 32 | slot).  A particle
// without contacts gets its wall collision here; the others get it after their
// binary collisions.
// MODE: CT_ALL, the collision stage's contacts; CT_ROWS, the rows and degrees
// of every particle and nothing else (no wall pass, marks, counters or flags),
// for the pair listing.
constexpr int CT_ALL = 0, CT_ROWS = 2;
template <int P, int W = CONTACT_W, int MODE = CT_ALL>
__device__ __forceinline__ void contacts_body(const int bidx, const int gdim, Parts<typename Prec<P>::T> pt,
    const int32_t *__restrict__ cs, Consts<typename Prec<P>::T> k, Adj adj, int32_t *__restrict__ deg,
    int32_t *__restrict__ done, int32_t *ticket, int32_t *flags, long long *pair_part, long long *wall_part,
    int32_t *__restrict__ chunk_busy, int32_t *need_sweep, long long *__restrict__ roots,
    int32_t *__restrict__ rcount) {
  using T = typename Prec<P>::T;
  __shared__ long long sh[BLOCK / 64];
  __shared__ int shi[BLOCK / 64];
  const int s = bidx * BLOCK + threadIdx.x;
  long long fwd = 0, nwall = 0;
  bool cand = false;  // has contacts, all with higher indices: a possible cluster root
  bool by_wall_pass = true;
  if (MODE != CT_ROWS && s == 0) {
    *ticket = 0;
    *need_sweep = 0;
  }
  if (s < k.npart) {
    const int key = pt.key[s];
    const int id = pt.pid[s];
    const T x = pt.px[s], y = pt.py[s];
    int cx, cy;
    cell_xy(k, key, cx, cy);
    // velocity for the wall pass of a contact-free particle: only a particle in a
    // cell next to a wall can need it
    const bool by_wall = (!k.per_x && (cx == 0 || cx == k.nx - 1)) || (!k.per_y && (cy == 0 || cy == k.ny - 1));
    T vx0 = (T)0, vy0 = (T)0;
    if (by_wall) {
      vx0 = pt.vx[s];
      vy0 = pt.vy[s];
    }
    const T dd = k.d * k.d;
    const AdjRow row = adj.row(s);
    // The particle's own row of cells (its cell and the cells left and right of
    // it) is one slot range around s, so the W slots on each side are
    // loaded now, before the cell starts arrive; the ones inside the row's
    // range are tested from registers.
    T wx[2 * W], wy[2 * W];
    int wid[2 * W];
#pragma unroll
    for (int j = 0; j < 2 * W; ++j) {
      const int t = min(max(j < W ? s - W + j : s + 1 + (j - W), 0), k.npart - 1);
      wx[j] = ldu(pt.px, t);
      wy[j] = ldu(pt.py, t);
      wid[j] = ldu(pt.pid, t);
    }
    // Pass 1 keeps the first CONTACT_REG contacts sorted in registers (no
    // stores while scanning, so candidate loads overlap); a particle with more
    // contacts is scanned again and its list built in memory.
    long long r[CONTACT_REG];
    int cnt = 0;
    bool over = false;
    // candidate ranges: the three cells of each neighbour row are one slot
    // range away from a periodic seam; the column offset of a candidate follows
    // from the cell starts.  All starts are loaded first.
    const bool inner_x = cx >= 1 && cx + 1 < k.nx;
    // A partner lies within d of the particle, so only the columns and rows of
    // cells that come within d of its position can hold one: with d <= 1/2
    // two of the three in each direction.  The margin keeps every candidate
    // whose rounded distance test could pass (rounding of a separation is
    // below 1e-6 at any lattice size the library accepts).
    const T fx = Pos<P>::G ? x - (T)cx : x, fy = Pos<P>::G ? y - (T)cy : y;  // position in the cell
    const T margin = (T)1e-5;
    const bool use_l = fx < k.d + margin, use_r = fx > (T)1 - k.d - margin;
    const bool use_b = fy < k.d + margin, use_t = fy > (T)1 - k.d - margin;
    int rlo[3], rm1[3], rm2[3], rhi[3];
#pragma unroll
    for (int rw = 0; rw < 3; ++rw) {
      int yy = cy + rw - 1;
      bool ok = rw == 0 ? use_b : (rw == 2 ? use_t : true);
      if (yy < 0 || yy >= k.ny) {
        ok = ok && k.per_y != 0;
        yy = wrap_i(yy, k.ny);
      }
      const int c0 = yy * k.nx + cx - 1;
      if (ok && inner_x) {
        rm1[rw] = ldu(cs, c0 + 1);
        rm2[rw] = ldu(cs, c0 + 2);
        rlo[rw] = use_l ? ldu(cs, c0) : rm1[rw];
        rhi[rw] = use_r ? ldu(cs, c0 + 3) : rm2[rw];
      } else {  // a row not needed or beyond a wall (empty), or a seam column walked cell by cell below
        rlo[rw] = rm1[rw] = rm2[rw] = rhi[rw] = 0;
      }
    }
    auto scan = [&](auto &&hit) {
      auto test = [&](int t, int ox, int oy) {
        if (t == s) return;
        T dx, dy;
        Pos<P>::sep_nb(k, ox, oy, x, y, pt.px[t], pt.py[t], dx, dy);
        if (dx * dx + dy * dy <= dd) hit(t, pt.pid[t]);
      };
      if (inner_x) {
        // one flattened pass over the three rows' ranges, CONTACT_CH candidates
        // at a time: their positions and indices are all loaded before any is
        // tested.  Candidate q of the flattened range is slot q + sh_r in row r.
        const int n0 = rhi[0] - rlo[0], n01 = n0 + rhi[1] - rlo[1];
        const int tot = n01 + rhi[2] - rlo[2];  // >= 1: the particle's own cell
        const int sh0 = rlo[0], sh1 = rlo[1] - n0, sh2 = rlo[2] - n01;
        // column boundaries as plain values (selected per candidate, not indexed)
        const int a0 = rm1[0], a1 = rm1[1], a2 = rm1[2], b0 = rm2[0], b1 = rm2[1], b2 = rm2[2];
        for (int q0 = 0; q0 < tot; q0 += CONTACT_CH) {
          int tt[CONTACT_CH], ox[CONTACT_CH], oy[CONTACT_CH], ids[CONTACT_CH];
          T xs[CONTACT_CH], ys[CONTACT_CH];
#pragma unroll
          for (int j = 0; j < CONTACT_CH; ++j) {
            const int q = min(q0 + j, tot - 1);  // past the end: repeat the last candidate
            const bool r0 = q < n0, r1 = q < n01;
            const int t = q + (r0 ? sh0 : (r1 ? sh1 : sh2));
            const int m1 = r0 ? a0 : (r1 ? a1 : a2), m2 = r0 ? b0 : (r1 ? b1 : b2);
            tt[j] = t;
            ox[j] = t < m1 ? -1 : (t < m2 ? 0 : 1);
            oy[j] = r0 ? -1 : (r1 ? 0 : 1);
            xs[j] = ldu(pt.px, t);
            ys[j] = ldu(pt.py, t);
            ids[j] = ldu(pt.pid, t);
          }
#pragma unroll
          for (int j = 0; j < CONTACT_CH; ++j) {
            if (q0 + j < tot && tt[j] != s) {
              T dx, dy;
              Pos<P>::sep_nb(k, ox[j], oy[j], x, y, xs[j], ys[j], dx, dy);
              if (dx * dx + dy * dy <= dd) hit(tt[j], ids[j]);
            }
          }
        }
      } else {
        for (int oy = -1; oy <= 1; ++oy) {
          int yy = cy + oy;
          if (yy < 0 || yy >= k.ny) {
            if (!k.per_y) continue;
            yy = wrap_i(yy, k.ny);
          }
          const int rb = yy * k.nx;
          for (int ox = -1; ox <= 1; ++ox) {
            int xx = cx + ox;
            if (xx < 0 || xx >= k.nx) {
              if (!k.per_x) continue;
              xx = wrap_i(xx, k.nx);
            }
            const int c = rb + xx;
            for (int t = cs[c]; t < cs[c + 1]; ++t) test(t, ox, oy);
          }
        }
      }
    };
    // Pass 1 over a row of cells away from a periodic seam: the window slots
    // inside the own row's range from registers, then the rest of the three
    // ranges (row below, own row left and right of the window, row above),
    // CONTACT_CH candidates at a time.
    auto first_scan = [&](auto &&hit) {
      if (!inner_x) {
        scan(hit);
        return;
      }
      const int lo1 = rlo[1], hi1 = rhi[1], a1 = rm1[1], b1 = rm2[1];
#pragma unroll
      for (int j = 0; j < 2 * W; ++j) {
        const int t = j < W ? s - W + j : s + 1 + (j - W);
        if (t >= lo1 && t < hi1) {
          T dx, dy;
          Pos<P>::sep_nb(k, t < a1 ? -1 : (t < b1 ? 0 : 1), 0, x, y, wx[j], wy[j], dx, dy);
          if (dx * dx + dy * dy <= dd) hit(t, wid[j]);
        }
      }
      const int mlo = max(lo1, s + W + 1);
      const int n0 = rhi[0] - rlo[0], n1 = n0 + max(0, min(hi1, s - W) - lo1);
      const int n2 = n1 + max(0, hi1 - mlo), tot = n2 + rhi[2] - rlo[2];
      const int sh0 = rlo[0], sh1 = lo1 - n0, sh2 = mlo - n1, sh3 = rlo[2] - n2;
      const int a0 = rm1[0], a2 = rm1[2], b0 = rm2[0], b2 = rm2[2];
      for (int q0 = 0; q0 < tot; q0 += CONTACT_CH) {
        int tt[CONTACT_CH], ox[CONTACT_CH], oy[CONTACT_CH], ids[CONTACT_CH];
        T xs[CONTACT_CH], ys[CONTACT_CH];
#pragma unroll
        for (int j = 0; j < CONTACT_CH; ++j) {
          const int q = min(q0 + j, tot - 1);  // past the end: repeat the last candidate
          const bool r0 = q < n0, r1 = q < n1, r2 = q < n2;
          const int t = q + (r0 ? sh0 : (r1 ? sh1 : (r2 ? sh2 : sh3)));
          const int m1 = r0 ? a0 : (r2 ? a1 : a2), m2 = r0 ? b0 : (r2 ? b1 : b2);
          tt[j] = t;
          ox[j] = t < m1 ? -1 : (t < m2 ? 0 : 1);
          oy[j] = r0 ? -1 : (r2 ? 0 : 1);
          xs[j] = ldu(pt.px, t);
          ys[j] = ldu(pt.py, t);
          ids[j] = ldu(pt.pid, t);
        }
#pragma unroll
        for (int j = 0; j < CONTACT_CH; ++j) {
          if (q0 + j < tot) {
            T dx, dy;
            Pos<P>::sep_nb(k, ox[j], oy[j], x, y, xs[j], ys[j], dx, dy);
            if (dx * dx + dy * dy <= dd) hit(tt[j], ids[j]);
          }
        }
      }
    };
    first_scan([&](int t, int tid) {
      if (tid > id) ++fwd;
      if (cnt < CONTACT_REG) {
        const long long e = ((long long)tid << 32) | (unsigned)t;
        bool placed = false;
#pragma unroll
        for (int u = CONTACT_REG - 1; u >= 0; --u)
          if (!placed && u <= cnt) {
            if (u > 0 && r[u - 1] > e) {
              r[u] = r[u - 1];
            } else {
              r[u] = e;
              placed = true;
            }
          }
      }
      ++cnt;
    });
    if (cnt <= CONTACT_REG) {
#pragma unroll
      for (int u = 0; u < CONTACT_REG; ++u)
        if (u < cnt) row[u] = r[u];
    } else {
      int m = 0;
      scan([&](int t, int tid) {
        if (m == KMAX) {
          over = true;
          return;
        }
        const long long e = ((long long)tid << 32) | (unsigned)t;
        int j = m;
        while (j > 0 && row[j - 1] > e) {
          row[j] = row[j - 1];
          --j;
        }
        row[j] = e;
        ++m;
      });
      cnt = m;
    }
    deg[s] = cnt;
    if constexpr (MODE == CT_ROWS) {
      fwd = 0;
      by_wall_pass = false;
    } else {
      if (over) atomicOr(&flags[FLAG_CAPACITY], 1);
      if (cnt > 0) cand = (int)((cnt <= CONTACT_REG ? r[0] : row[0]) >> 32) > id;
      done[s] = 0;
      if (cnt > 0) chunk_busy[id / RES_CHUNK] = 1;  // the resolution visits this chunk of indices
    }
    if (by_wall_pass && cnt == 0 && by_wall) {  // no binary collision: the wall pass can run now
      const int h = Pos<P>::walls(k, cx, cy, x, y, vx0, vy0);
      if (h) {
        pt.vx[s] = vx0;
        pt.vy[s] = vy0;
        nwall += h;
      }
    }
  }
  if constexpr (MODE == CT_ROWS) return;  // uniform
  // candidate roots of this workgroup, compacted to the front of its segment
  int nc;
  const int off = block_excl_scan(cand ? 1 : 0, shi, nc);
  if (cand) roots[(size_t)bidx * BLOCK + off] = ((long long)pt.pid[s] << 32) | (unsigned)s;
  long long t, tw;
  block_sum2(fwd, nwall, sh, t, tw);
  if (threadIdx.x == 0) {
    pair_part[bidx] = t;
    wall_part[bidx] = tw;
    rcount[bidx] = nc;
  }
}
template <int P, int MODE = CT_ALL>
__global__ __launch_bounds__(BLOCK) LBDPS_WAVES8 void k_contacts(Parts<typename Prec<P>::T> pt, const int32_t *__restrict__ cs,
                                                    Consts<typename Prec<P>::T> k, Adj adj,
                                                    int32_t *__restrict__ deg, int32_t *__restrict__ done,
                                                    int32_t *ticket, int32_t *flags, long long *pair_part,
                                                    long long *wall_part, int32_t *__restrict__ chunk_busy,
                                                    int32_t *need_sweep, long long *__restrict__ roots,
                                                    int32_t *__restrict__ rcount) {
  contacts_body<P, CONTACT_W, MODE>(xcd_block<XCD_RUN_CONTACTS>(blockIdx.x, gridDim.x), gridDim.x, pt, cs, k, adj, deg, done, ticket, flags, pair_part, wall_part, chunk_busy,
      need_sweep, roots, rcount);
}
// Grids whose workgroups are all resident at once (CONTACTS_SMALL_MAX): a wider
// early-loaded window at six waves per SIMD, since latency rather than the
// number of waves in flight bounds such a launch.
constexpr int CONTACTS_SMALL_MAX = 1536;
template <int P, int MODE = CT_ALL>
__global__ __launch_bounds__(BLOCK) LBDPS_WAVES6 void k_contacts_small(Parts<typename Prec<P>::T> pt,
    const int32_t *__restrict__ cs, Consts<typename Prec<P>::T> k, Adj adj, int32_t *__restrict__ deg,
    int32_t *__restrict__ done, int32_t *ticket, int32_t *flags, long long *pair_part, long long *wall_part,
    int32_t *__restrict__ chunk_busy, int32_t *need_sweep, long long *__restrict__ roots,
    int32_t *__restrict__ rcount) {
  contacts_body<P, CONTACT_W_SMALL, MODE>(xcd_block<XCD_RUN_CONTACTS>(blockIdx.x, gridDim.x), gridDim.x, pt, cs, k, adj,
                                    deg, done, ticket, flags, pair_part, wall_part, chunk_busy, need_sweep, roots,
                                    rcount);
}

// ------------------------------------------------------------------ A7: collision resolution (Eqs. 17-18) and walls
// Sequential semantics: pairs (i, j), i < j, processed in lexicographic order,
// each with the current velocities.  A pair touches only its two particles, so
// the result is fixed by the order of each particle's own pairs.  Each
// particle's pairs in that order are exactly its neighbours by ascending index;
// done[s] counts how many of them are finished.  The owner of a pair is its
// lower-index particle; it fires the pair once both particles have finished
// all earlier pairs.  Every wait is for a lexicographically earlier pair, whose
// owner has a lower particle index; workgroups take particle ranges in the
// order they start (atomic ticket), so the owner of the earliest unfinished
// pair is always running and the sweep always progresses.  Waits are bounded
// by spin_limit polls; exceeding it latches FLAG_STALL and the wave exits.
// Binary collision of slots s (lower particle index) and t, Eqs. 17-18 with the
// current velocities; the pair collides only if (P_s - P_t).(v_s - v_t) < 0.
// The collision of two particles given by value: separation (dx, dy) = P_s - P_t
// and velocities; returns whether they approach, and then the new velocities.
// Every operation is one IEEE operation in the arithmetic type, the two
// divisions correctly rounded (not the hardware reciprocal) in every
// precision, so that the outcome is fixed by the arithmetic type alone: in
// FP32 it is the same float computation step for step on any IEEE machine.
template <int P>
__device__ __forceinline__ bool pair_core(const Consts<typename Prec<P>::T> &k, typename Prec<P>::T dx,
                                          typename Prec<P>::T dy, typename Prec<P>::T &vix, typename Prec<P>::T &viy,
                                          typename Prec<P>::T &vjx, typename Prec<P>::T &vjy) {
  using T = typename Prec<P>::T;
  const T dvx = vix - vjx, dvy = viy - vjy;
  const T dot = dvx * dx + dvy * dy;
  if (!(dot < (T)0)) return false;
  const T r2 = dx * dx + dy * dy;
  const T q0 = (k.one_e * dot) / r2;
  const T ci = (q0 * k.m) / k.msum;
  const T cj = ci;  // m_i / (m_i + m_j) = m_j / (m_i + m_j): one mass
  vix = vix - ci * dx;
  viy = viy - ci * dy;
  vjx = vjx + cj * dx;
  vjy = vjy + cj * dy;
  return true;
}

template <int P>
__device__ __forceinline__ bool pair_collide(const Consts<typename Prec<P>::T> &k, Parts<typename Prec<P>::T> &pt,
                                             int s, int t) {
  using T = typename Prec<P>::T;
  T dx, dy;
  Pos<P>::sep(k, pt.key[s], pt.px[s], pt.py[s], pt.key[t], pt.px[t], pt.py[t], dx, dy);
  T vix = pt.vx[s], viy = pt.vy[s], vjx = pt.vx[t], vjy = pt.vy[t];
  if (!pair_core<P>(k, dx, dy, vix, viy, vjx, vjy)) return false;
  pt.vx[s] = vix;
  pt.vy[s] = viy;
  pt.vx[t] = vjx;
  pt.vy[t] = vjy;
  return true;
}

template <int P>
__device__ __forceinline__ int wall_pass(const Consts<typename Prec<P>::T> &k, Parts<typename Prec<P>::T> &pt, int s) {
  using T = typename Prec<P>::T;
  T vx = pt.vx[s], vy = pt.vy[s];
  const int key = pt.key[s];
  const int h = Pos<P>::walls_key(k, key, pt.px[s], pt.py[s], vx, vy);
  if (h) {
    pt.vx[s] = vx;
    pt.vy[s] = vy;
  }
  return h;
}

// Contact clusters (connected components of the contact graph) are independent:
// a pair only touches its two particles, so resolving every cluster's pairs in
// lexicographic order gives the sequential sweep's result bit for bit.  The
// contact kernel lists, per workgroup, the particles whose neighbours all have
// higher indices: every cluster's lowest index is among them.  A lane takes one
// such candidate, gathers its cluster breadth-first and gives up as soon as it
// meets a lower index (the cluster belongs to another candidate).  Otherwise it
// orders the members by index, applies the pairs in order, runs the wall pass
// of each member and marks them finished (done = number of contacts).  No lane
// waits for another.
//
// The cluster is gathered into CL_LDS entries of LDS; a larger one is queued
// for the whole workgroup (below), and one the queue cannot take is left to
// the ordered sweep of k_resolve.  Each workgroup takes the candidate lists of
// a run of contact-kernel workgroups and deals their candidates out to its
// lanes densely.
constexpr int CL_LDS = 8;
constexpr int RC_LISTS = 1;           // candidate lists per resolution workgroup (default)
constexpr int RC_GROUPS_MAX = 1 << 30;  // most resolution workgroups (default: no limit)

struct LdsColumn {  // entry i of a lane's column of a [CL_LDS][BLOCK] LDS array
  long long *p;
  __device__ long long &operator[](int i) const { return p[i * BLOCK]; }
};

// A gathered member is stored as (index << 32 | pos << 29 | slot): pos is its
// place in the breadth-first order (slots are below 2^29), so ordering the
// entries orders the members by index and each keeps its place.  The cluster's
// contacts are kept as an 8 x 8 bit matrix over those places (bit 8 a + b:
// places a and b touch); every contact of a member is inside the cluster, so
// the matrix holds each member's whole neighbour list.
static_assert(CL_LDS <= 8, "places of the members fit in three bits");
__device__ __forceinline__ unsigned long long cl_bit(int a, int b) { return 1ull << (8 * a + b); }

// Gathers the cluster of candidate slot s (index g) into q[0 .. m) and its
// contacts into A; returns m, 0 if a member has a lower index than g, and -1
// if the cluster has more than cap (<= CL_LDS) members.  Members are expanded
// two at a time, so the rows of both are loaded together.  The members' slots
// are also kept in registers, where the membership test looks them up.
template <class Row>
__device__ __forceinline__ int gather_cluster(Row q, int cap, int s, int g, Adj adj,
                                              const int32_t *__restrict__ deg, unsigned long long &A) {
  q[0] = ((long long)g << 32) | (unsigned)s;
  A = 0;
  int m = 1;
  int sl[CL_LDS];  // slot of the member at each place, -1 past m
#pragma unroll
  for (int i = 0; i < CL_LDS; ++i) sl[i] = i == 0 ? s : -1;
  // adds the contacts of the member at place h; false when the candidate gives up
  auto expand = [&](int h, const AdjRow &ru, int du, const Dense4 &e4, int &res) {
    for (int a = 0; a < du; ++a) {
      const long long e = a < ADJ_IN ? e4.get(a) : ru[a];
      if ((int)(e >> 32) < g) {
        res = 0;
        return false;
      }
      const int es = (int)(e & 0x1fffffffll);
      int p = -1;
#pragma unroll
      for (int i = 0; i < CL_LDS; ++i)
        if (sl[i] == es) p = i;
      if (p < 0) {
        if (m == cap) {
          res = -1;
          return false;
        }
        p = m;
        q[m] = e | ((long long)m << 29);
#pragma unroll
        for (int i = 1; i < CL_LDS; ++i)
          if (i == m) sl[i] = es;
        ++m;
      }
      A |= cl_bit(h, p) | cl_bit(p, h);
    }
    return true;
  };
  for (int head = 0; head < m;) {
    const bool two = head + 1 < m;
    int u0 = s, u1 = s;
#pragma unroll
    for (int i = 1; i < CL_LDS; ++i) {
      if (i == head) u0 = sl[i];
      if (i == head + 1) u1 = sl[i];
    }
    if (!two) u1 = u0;
    const AdjRow r0 = adj.row(u0), r1 = adj.row(u1);
    const int d0 = min(ldu(deg, u0), KMAX), d1 = two ? min(ldu(deg, u1), KMAX) : 0;
    // the dense parts of both rows
    const Dense4 f(r0.a), h(r1.a);
    int res = 0;
    if (!expand(head, r0, d0, f, res)) return res;
    if (two && !expand(head + 1, r1, d1, h, res)) return res;
    head += two ? 2 : 1;
  }
  return m;
}

// Orders the m gathered entries by index: all are read at once and each is
// written to its rank among them (the indices are distinct), so no chain of
// dependent LDS accesses as an insertion sort would make.
template <class Row> __device__ __forceinline__ void sort_members(Row q, int m) {
  long long e[CL_LDS];
#pragma unroll
  for (int i = 0; i < CL_LDS; ++i) e[i] = i < m ? q[i] : 0x7fffffffffffffffll;
#pragma unroll
  for (int i = 0; i < CL_LDS; ++i) {
    int r = 0;
#pragma unroll
    for (int j = 0; j < CL_LDS; ++j) r += e[j] < e[i];
    if (i < m) q[r] = e[i];
  }
}

// Orders the gathered members by index and applies the cluster's pairs in
// lexicographic order: member i (ascending) meets its higher-index neighbours
// in ascending order.  Every pair with it as the higher index came before, and
// none follows, so its wall pass runs right after its own pairs.  The
// neighbours come from the contact matrix, so no row is read again, and the
// records of all members are loaded in one round (registers indexed by the
// members' places in index order), so the pairs run with no memory round
// trip between them.
template <int P, class Row>
__device__ __forceinline__ void resolve_cluster(Row q, int m, unsigned long long A,
                                                const Consts<typename Prec<P>::T> &k,
                                                Parts<typename Prec<P>::T> &pt, int32_t *done, long long &ncoll,
                                                long long &nwall) {
  using T = typename Prec<P>::T;
  sort_members(q, m);
  int pl[CL_LDS], kk[CL_LDS];
  T xx[CL_LDS], yy[CL_LDS], vx[CL_LDS], vy[CL_LDS];
#pragma unroll
  for (int i = 0; i < CL_LDS; ++i) {
    pl[i] = 0;
    if (i < m) {
      const long long qi = q[i];
      const int u = (int)(qi & 0x1fffffffll);
      pl[i] = (int)((qi >> 29) & 7);
      kk[i] = ldu(pt.key, u);
      xx[i] = ldu(pt.px, u);
      yy[i] = ldu(pt.py, u);
      vx[i] = ldu(pt.vx, u);
      vy[i] = ldu(pt.vy, u);
    }
  }
#pragma unroll
  for (int i = 0; i < CL_LDS; ++i) {
    if (i < m) {
      const unsigned nbr = (unsigned)(A >> (8 * pl[i])) & 0xffu;  // places of its neighbours
#pragma unroll
      for (int j = i + 1; j < CL_LDS; ++j) {
        if (j < m && ((nbr >> pl[j]) & 1u)) {
          T dx, dy;
          Pos<P>::sep(k, kk[i], xx[i], yy[i], kk[j], xx[j], yy[j], dx, dy);
          ncoll += pair_core<P>(k, dx, dy, vx[i], vy[i], vx[j], vy[j]);
        }
      }
      nwall += Pos<P>::walls_key(k, kk[i], xx[i], yy[i], vx[i], vy[i]);
      const int u = (int)(q[i] & 0x1fffffffll);  // the slot again from LDS rather than held
      pt.vx[u] = vx[i];
      pt.vy[u] = vy[i];
      done[u] = __builtin_popcount(nbr) | DONE_WHOLE;  // its contacts, all inside the cluster
    }
  }
}

// A cluster of more than CL_LDS members is resolved by a group of threads with
// everything in LDS: breadth-first gathering with an open-addressing set of
// member slots, a bitonic sort by index, the lexicographic pair list built
// with a group scan, the pairs applied in order by one thread on the members'
// LDS copies, then the wall pass of every member in parallel.  A group is one
// wavefront (clusters of up to 64 members and 256 pairs; the four wavefronts of
// a workgroup take queued clusters in parallel) or the whole workgroup (up to
// 256 members and 1024 pairs, for clusters a wavefront could not hold).  A
// cluster beyond that is left to the ordered sweep.
constexpr int BIG_LIST = 64;  // clusters queued per workgroup for the group paths
constexpr int WAVE = 64;

template <int G> struct Group {  // G = BLOCK: the workgroup; G = WAVE: one wavefront
  static_assert(G == BLOCK || G == WAVE, "group size");
  __device__ static int rank() { return G == BLOCK ? (int)threadIdx.x : (int)(threadIdx.x & (WAVE - 1)); }
  __device__ static void sync() {
    if constexpr (G == BLOCK) {
      __syncthreads();
    } else {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  // Exclusive scan of one int per thread over the group, and the group total.
  __device__ static int excl_scan(int v, int *shi, int &total) {
    if constexpr (G == BLOCK) {
      return block_excl_scan(v, shi, total);
    } else {
      const int lane = rank();
      int inc = v;
      for (int o = 1; o < WAVE; o <<= 1) {
        const int u = __shfl_up(inc, o, WAVE);
        if (lane >= o) inc += u;
      }
      total = __shfl(inc, WAVE - 1, WAVE);
      return inc - v;
    }
  }
};

template <int P, int G> struct ClusterLds {
  using T = typename Prec<P>::T;
  static constexpr int MAX = G, HASH = 2 * G, PAIRS = 4 * G;
  long long q[MAX];
  int hslot[HASH];
  short hidx[HASH];
  int key[MAX];
  T px[MAX], py[MAX], vx[MAX], vy[MAX];
  unsigned pairs[PAIRS];
  int m, notroot, over;

  __device__ static int hash(int slot) { return (int)(((unsigned)slot * 2654435761u) >> 20) & (HASH - 1); }
  // Insert slot into the set; returns 1 if it was new, 0 if present, -1 if full.
  __device__ int insert(int slot) {
    int h = hash(slot);
    for (int probe = 0; probe < HASH; ++probe) {
      const int old = atomicCAS(&hslot[h], -1, slot);
      if (old == -1) return 1;
      if (old == slot) return 0;
      h = (h + 1) & (HASH - 1);
    }
    return -1;
  }
  __device__ int find(int slot) const {
    int h = hash(slot);
    for (int probe = 0; probe < HASH; ++probe) {
      const int v = hslot[h];
      if (v == slot) return h;
      if (v == -1) return -1;
      h = (h + 1) & (HASH - 1);
    }
    return -1;
  }
};

// Resolution of the cluster of candidate slot s0 (index g) by group G; every
// thread of the group calls it.  Returns 0 when resolved, 1 when a member has
// a lower index than g (another candidate owns the cluster), 2 when the cluster
// exceeds the group's capacity (nothing was changed).
template <int P, int G>
__device__ int resolve_group(ClusterLds<P, G> &B, int *shi, int s0, int g, const Consts<typename Prec<P>::T> &k,
                             Parts<typename Prec<P>::T> &pt, Adj adj, const int32_t *__restrict__ deg, int32_t *done,
                             long long &ncoll, long long &nwall) {
  using T = typename Prec<P>::T;
  using Gr = Group<G>;
  constexpr int MAX = ClusterLds<P, G>::MAX;
  const int tid = Gr::rank();
  for (int i = tid; i < ClusterLds<P, G>::HASH; i += G) B.hslot[i] = -1;
  if (tid == 0) {
    B.q[0] = ((long long)g << 32) | (unsigned)s0;
    B.m = 1;
    B.notroot = 0;
    B.over = 0;
  }
  Gr::sync();
  if (tid == 0) B.insert(s0);
  Gr::sync();
  // level-synchronous breadth-first gathering
  int h0 = 0;
  for (;;) {
    const int h1 = min(B.m, MAX);
    const bool stop = h0 >= h1 || B.notroot || B.over;
    Gr::sync();
    if (stop) break;
    for (int t = h0 + tid; t < h1; t += G) {
      const int u = (int)(B.q[t] & 0xffffffffll);
      const AdjRow ru = adj.row(u);
      const int du = min(deg[u], KMAX);
      for (int a = 0; a < du; ++a) {
        const long long e = ru[a];
        if ((int)(e >> 32) < g) {
          B.notroot = 1;  // a lower index: the cluster belongs to another candidate
          break;
        }
        const int r = B.insert((int)(e & 0xffffffffll));
        if (r < 0) {
          B.over = 1;
          break;
        }
        if (r == 1) {
          const int pos = atomicAdd(&B.m, 1);
          if (pos < MAX) B.q[pos] = e;
          else B.over = 1;
        }
      }
    }
    Gr::sync();
    h0 = h1;
  }
  if (B.notroot) return 1;  // uniform: read after the loop's last barrier
  if (B.over) return 2;
  const int m = B.m;
  // bitonic sort of q[0 .. MAX) by (index, slot), padded past m
  if (tid >= m) B.q[tid] = 0x7fffffffffffffffll;
  Gr::sync();
  for (int len = 2; len <= MAX; len <<= 1)
    for (int st = len >> 1; st > 0; st >>= 1) {
      const int j = tid ^ st;
      if (j > tid) {
        const long long a = B.q[tid], b = B.q[j];
        const bool up = (tid & len) == 0;
        if ((a > b) == up) {
          B.q[tid] = b;
          B.q[j] = a;
        }
      }
      Gr::sync();
    }
  // member copies, slot -> sorted index, pairs (i, j), i < j, per member
  const bool mem = tid < m;
  const int u = mem ? (int)(B.q[tid] & 0xffffffffll) : 0;
  const int gu = mem ? (int)(B.q[tid] >> 32) : 0;
  int cnt = 0;
  if (mem) {
    B.hidx[B.find(u)] = (short)tid;
    B.key[tid] = pt.key[u];
    B.px[tid] = pt.px[u];
    B.py[tid] = pt.py[u];
    B.vx[tid] = pt.vx[u];
    B.vy[tid] = pt.vy[u];
    const AdjRow ru = adj.row(u);
    const int du = min(deg[u], KMAX);
    for (int a = 0; a < du; ++a) cnt += (int)(ru[a] >> 32) > gu;
  }
  int npairs;
  const int off = Gr::excl_scan(cnt, shi, npairs);
  if (npairs > ClusterLds<P, G>::PAIRS) return 2;
  Gr::sync();  // every member's slot -> index entry is written
  if (mem) {
    const AdjRow ru = adj.row(u);
    const int du = min(deg[u], KMAX);
    int w = off;
    for (int a = 0; a < du; ++a) {
      const long long e = ru[a];
      if ((int)(e >> 32) > gu) B.pairs[w++] = ((unsigned)tid << 16) | (unsigned)B.hidx[B.find((int)(e & 0xffffffffll))];
    }
  }
  Gr::sync();
  if (tid == 0) {  // the pairs in lexicographic order, on the LDS copies
    for (int q = 0; q < npairs; ++q) {
      const int i = (int)(B.pairs[q] >> 16), j = (int)(B.pairs[q] & 0xffffu);
      T dx, dy;
      Pos<P>::sep(k, B.key[i], B.px[i], B.py[i], B.key[j], B.px[j], B.py[j], dx, dy);
      T vix = B.vx[i], viy = B.vy[i], vjx = B.vx[j], vjy = B.vy[j];
      if (pair_core<P>(k, dx, dy, vix, viy, vjx, vjy)) {
        B.vx[i] = vix;
        B.vy[i] = viy;
        B.vx[j] = vjx;
        B.vy[j] = vjy;
        ++ncoll;
      }
    }
  }
  Gr::sync();
  if (mem) {
    T vx = B.vx[tid], vy = B.vy[tid];
    const int key = B.key[tid];
    nwall += Pos<P>::walls_key(k, key, B.px[tid], B.py[tid], vx, vy);
    pt.vx[u] = vx;
    pt.vy[u] = vy;
    done[u] = deg[u] | DONE_WHOLE;
  }
  Gr::sync();
  return 0;
}

template <int P>
__device__ __forceinline__ void resolve_clusters_body(const int bidx, const int gdim, Parts<typename Prec<P>::T> pt,
    Adj adj, const int32_t *__restrict__ deg, int32_t *done, Consts<typename Prec<P>::T> k, int32_t *need_sweep,
    long long *coll_part, long long *wall_part, const long long *__restrict__ roots,
    const int32_t *__restrict__ rcount, int nlists, const int32_t *nroots = nullptr) {
  __shared__ long long sh[BLOCK / 64];
  __shared__ int shi[BLOCK / 64];
  __shared__ int pre[BLOCK + 1];
  __shared__ long long bigc[BIG_LIST], hugec[BIG_LIST];
  __shared__ int nbig, nhuge;
  // the per-lane gathering area, reused afterwards for the group paths
  __shared__ union {
    long long qs[CL_LDS * BLOCK];
    ClusterLds<P, WAVE> wave[BLOCK / WAVE];
    ClusterLds<P, BLOCK> big;
  } U;
  long long *const qs = U.qs;
  if (threadIdx.x == 0) {
    nbig = 0;
    nhuge = 0;
  }
  // candidate lists [b0, b0 + nb) of the contact kernel's workgroups
  const int per = (nlists + gdim - 1) / gdim;  // <= BLOCK (host grid choice)
  const int b0 = bidx * per;
  const int nb = max(0, min(nlists - b0, per));
  int tot;
  // a contact row over its capacity leaves the contact graph incomplete: the
  // resolution is skipped and the step reports LBDPS_E_CAPACITY
  const bool overflow = __hip_atomic_load(&k.flags[FLAG_CAPACITY], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
  // list j holds rcount[j] candidates, or, with one compact list of *nroots
  // (the tile kernel's), its j-th run of BLOCK
  // (the counts are loaded alongside the flag, not after it)
  int c = 0;
  if ((int)threadIdx.x < nb)
    c = nroots ? min(max(*nroots - (b0 + (int)threadIdx.x) * BLOCK, 0), BLOCK) : rcount[b0 + threadIdx.x];
  if (overflow) c = 0;
  const int o = block_excl_scan(c, shi, tot);
  if (tot == 0) {  // no candidate roots in these lists (uniform: the scan's total)
    if (threadIdx.x == 0) {
      coll_part[bidx] = 0;
      wall_part[bidx] = 0;
    }
    return;
  }
  if ((int)threadIdx.x < nb) pre[threadIdx.x] = o;
  if (threadIdx.x == 0) pre[nb] = tot;
  __syncthreads();
  const LdsColumn ql{qs + threadIdx.x};
  long long ncoll = 0, nwall = 0;
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
    int m = gather_cluster(ql, CL_LDS, s, g, adj, deg, A);
    if (m > 0) {
      resolve_cluster<P>(ql, m, A, k, pt, done, ncoll, nwall);
    } else if (m < 0) {
      const int slot = atomicAdd(&nbig, 1);  // the workgroup resolves it below
      if (slot < BIG_LIST) bigc[slot] = r;
      else atomicOr(need_sweep, 1);  // queue full: the ordered sweep takes it
    }
  }
  __syncthreads();
  // queued clusters: one wavefront each, then the whole workgroup for those too large
  const int nb_big = min(nbig, BIG_LIST), wv = (int)threadIdx.x / WAVE;
  for (int c = wv; c < nb_big; c += BLOCK / WAVE) {
    const long long r = bigc[c];
    const int st = resolve_group<P, WAVE>(U.wave[wv], shi, (int)(r & 0xffffffffll), (int)(r >> 32), k, pt, adj, deg,
                                          done, ncoll, nwall);
    if (st == 2 && Group<WAVE>::rank() == 0) hugec[atomicAdd(&nhuge, 1)] = r;
  }
  __syncthreads();
  const int nb_huge = nhuge;
  for (int c = 0; c < nb_huge; ++c) {
    const long long r = hugec[c];
    const int st = resolve_group<P, BLOCK>(U.big, shi, (int)(r & 0xffffffffll), (int)(r >> 32), k, pt, adj, deg, done,
                                           ncoll, nwall);
    if (st == 2 && threadIdx.x == 0) atomicOr(need_sweep, 1);
  }
  long long tc, tw;
  block_sum2(ncoll, nwall, sh, tc, tw);
  if (threadIdx.x == 0) {
    coll_part[bidx] = tc;
    wall_part[bidx] = tw;
  }
}
template <int P>
__global__ __launch_bounds__(BLOCK) void k_resolve_clusters(Parts<typename Prec<P>::T> pt,
                                                            Adj adj,
                                                            const int32_t *__restrict__ deg, int32_t *done,
                                                            Consts<typename Prec<P>::T> k, int32_t *need_sweep,
                                                            long long *coll_part, long long *wall_part,
                                                            const long long *__restrict__ roots,
                                                            const int32_t *__restrict__ rcount, int nlists,
                                                            const int32_t *nroots) {
  resolve_clusters_body<P>(xcd_block<XCD_RUN_CLUSTERS>(blockIdx.x, gridDim.x), gridDim.x, pt, adj, deg, done, k, need_sweep, coll_part, wall_part, roots,
      rcount, nlists, nroots);
}

// Position of particle index g in the neighbour list of slot t: the number of
// neighbours of t with a lower index (bounded by the list length).
__device__ __forceinline__ int row_position(Adj adj, const int32_t *deg, int t, int g) {
  const AdjRow rt = adj.row(t);
  const int n = min(deg[t], KMAX);
  int b = 0;
  while (b < n && (int)(rt[b] >> 32) < g) ++b;
  return b;
}


template <int P>
__device__ __forceinline__ void resolve_body(const int bidx, const int gdim, Parts<typename Prec<P>::T> pt,
    const int32_t *__restrict__ slot, Adj adj, const int32_t *__restrict__ deg, int32_t *done, int32_t *ticket,
    Consts<typename Prec<P>::T> k, int32_t *flags, long long *coll_part, long long *wall_part,
    int32_t *__restrict__ chunk_busy, int32_t *need_sweep) {
  using T = typename Prec<P>::T;
  __shared__ int s_ticket;
  // the tile kernel's compact root list is consumed: empty it for the next stage
  if (bidx == 0 && threadIdx.x == 0) need_sweep[1] = 0;
  __shared__ long long sh[BLOCK / 64];
  long long ncoll = 0, nwall = 0;
  unsigned spins = 0;
  // Chunks of RES_CHUNK particle indices are taken in increasing order from an
  // atomic ticket; chunks that hold no particle with a contact are skipped.
  const int nchunks = (k.npart + RES_CHUNK - 1) / RES_CHUNK;
  // every cluster was resolved whole, or a contact row overflowed (the
  // resolution is skipped): only clear the chunk marks
  if (!*need_sweep || __hip_atomic_load(&flags[FLAG_CAPACITY], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
    for (int i = bidx * BLOCK + threadIdx.x; i < nchunks; i += gdim * BLOCK) chunk_busy[i] = 0;
    if (threadIdx.x == 0) {
      coll_part[bidx] = 0;
      wall_part[bidx] = 0;
    }
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
    // This lane owns particle indices base + j BLOCK, j = 0 .. RES_ITEMS-1, taken
    // in increasing order; a later one is started only when the earlier is done.
    const int base = tk * RES_CHUNK + (int)threadIdx.x;
    int j = 0, g = base;
    int state = 2;  // 0: pair pending, 1: waiting for all pairs, 2: finished
    int s = 0, dg = 0, a = 0, t = 0, b = 0;
    AdjRow row{nullptr, nullptr};
    // Set up the next owned particle that has contacts (those without had
    // their wall pass in the contact kernel).
    auto next = [&]() {
      for (; j < RES_ITEMS; ++j) {
        g = base + j * BLOCK;
        if (g >= k.npart) {
          j = RES_ITEMS;
          break;
        }
        s = slot[g];
        dg = deg[s];
        // no contacts (wall pass in the contact kernel), or resolved whole with
        // its cluster; a particle whose pairs the sweep's lower partners have
        // all fired still takes its wall pass here (state 1)
        if (dg == 0 || done[s] >= DONE_WHOLE) continue;
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
          ncoll += pair_collide<P>(k, pt, s, t);
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
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          nwall += wall_pass<P>(k, pt, s);
          ++j;
          next();
          progressed = true;
        }
      }
      if (state != 2 && !progressed) {
        if (++spins > k.spin_limit) {
          atomicOr(&flags[FLAG_STALL], 1);
          state = 2;
          j = RES_ITEMS;
        } else {
          __builtin_amdgcn_s_sleep(1);
        }
      }
    }
  }
  const long long tc = block_sum_ll(ncoll, sh);
  const long long tw = block_sum_ll(nwall, sh);
  if (threadIdx.x == 0) {
    coll_part[bidx] = tc;
    wall_part[bidx] = tw;
  }
}
template <int P>
__global__ __launch_bounds__(BLOCK) void k_resolve(Parts<typename Prec<P>::T> pt, const int32_t *__restrict__ slot,
                                                   Adj adj, const int32_t *__restrict__ deg,
                                                   int32_t *done, int32_t *ticket, Consts<typename Prec<P>::T> k,
                                                   int32_t *flags, long long *coll_part, long long *wall_part,
                                                   int32_t *__restrict__ chunk_busy, int32_t *need_sweep) {
  resolve_body<P>(blockIdx.x, gridDim.x, pt, slot, adj, deg, done, ticket, k, flags, coll_part, wall_part, chunk_busy,
      need_sweep);
}

// ------------------------------------------------------------------ exclusive scan of int32


// Cell starts in one pass: the tile sums were accumulated while counting, so
// each workgroup adds the sums of all tiles before its own (a strided sum),
// scans its SCAN_TILE counts, writes cell_start and clears the counts.  A
// thread takes SCAN_ITEMS consecutive cells with 16-byte loads and stores, and
// one 64-bit workgroup scan carries both sums: the high word the tile sums
// before this tile, the low word this tile's counts (below 2^31, so no carry
// crosses into the high word).
__device__ __forceinline__ void scan_cells_body(const int bidx, const int gdim, int32_t *__restrict__ count,
    long long n, TileSums ts, int32_t *__restrict__ out, const int32_t *__restrict__ stay) {
  static_assert(SCAN_ITEMS == 8, "two 16-byte vectors per thread");
  __shared__ long long sh[BLOCK / 64];
  const int b = bidx;
  const long long e0 = (long long)b * SCAN_TILE + (long long)threadIdx.x * SCAN_ITEMS;
  const bool full = e0 + SCAN_ITEMS <= n;
  int vals[SCAN_ITEMS];
  if (full) {
    const int4 c0 = *(const int4 *)(count + e0), c1 = *(const int4 *)(count + e0 + 4);
    const int4 s0 = *(const int4 *)(stay + e0), s1 = *(const int4 *)(stay + e0 + 4);
    vals[0] = c0.x + s0.x;
    vals[1] = c0.y + s0.y;
    vals[2] = c0.z + s0.z;
    vals[3] = c0.w + s0.w;
    vals[4] = c1.x + s1.x;
    vals[5] = c1.y + s1.y;
    vals[6] = c1.z + s1.z;
    vals[7] = c1.w + s1.w;
  } else {
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) vals[j] = e0 + j < n ? count[e0 + j] + stay[e0 + j] : 0;
  }
  int sum = 0;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; ++j) sum += vals[j];
  int v = 0;
#pragma unroll 8
  for (int i = threadIdx.x; i < b; i += BLOCK) v += ts.tile[i];
  long long tot;
  const long long pre = block_excl_scan_ll(((long long)v << 32) | (unsigned)sum, sh, tot);
  const int base = (int)(tot >> 32);
  int o[SCAN_ITEMS];
  int run = base + (int)(pre & 0xffffffffll);
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; ++j) {
    o[j] = run;
    run += vals[j];
  }
  if (full) {
    *(int4 *)(out + e0) = make_int4(o[0], o[1], o[2], o[3]);
    *(int4 *)(out + e0 + 4) = make_int4(o[4], o[5], o[6], o[7]);
    *(int4 *)(count + e0) = make_int4(0, 0, 0, 0);
    *(int4 *)(count + e0 + 4) = make_int4(0, 0, 0, 0);
  } else {
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j)
      if (e0 + j < n) {
        out[e0 + j] = o[j];
        count[e0 + j] = 0;
      }
  }
  if (b == gdim - 1 && threadIdx.x == 0) out[n] = base + (int)(tot & 0xffffffffll);
}
__global__ __launch_bounds__(BLOCK) void k_scan_cells(int32_t *__restrict__ count, long long n, TileSums ts,
                                                      int32_t *__restrict__ out, const int32_t *__restrict__ stay) {
  scan_cells_body(xcd_block<XCD_RUN_SCAN>(blockIdx.x, gridDim.x), gridDim.x, count, n, ts, out, stay);
}

// Generic three-pass scan of n counts (reduce, top, apply), for scans whose
// tile sums nobody counted beforehand.  A full run of SCAN_ITEMS counts moves
// as two 16-byte vectors (the arrays are 256-byte aligned).
__device__ __forceinline__ bool scan_load8(const int32_t *__restrict__ in, long long e0, long long n, int v[8]) {
  if (e0 + SCAN_ITEMS <= n) {
    const int4 a = *(const int4 *)(in + e0), b = *(const int4 *)(in + e0 + 4);
    v[0] = a.x;
    v[1] = a.y;
    v[2] = a.z;
    v[3] = a.w;
    v[4] = b.x;
    v[5] = b.y;
    v[6] = b.z;
    v[7] = b.w;
    return true;
  }
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; ++j) v[j] = e0 + j < n ? in[e0 + j] : 0;
  return false;
}

__global__ __launch_bounds__(BLOCK) void k_scan_reduce(const int32_t *__restrict__ in, long long n,
                                                       int32_t *__restrict__ part) {
  static_assert(SCAN_ITEMS == 8, "two 16-byte vectors per thread");
  __shared__ int sh[BLOCK / 64];
  const long long base = (long long)blockIdx.x * SCAN_TILE + (long long)threadIdx.x * SCAN_ITEMS;
  int vals[SCAN_ITEMS];
  scan_load8(in, base, n, vals);
  int v = 0;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; ++j) v += vals[j];
  int total;
  block_excl_scan(v, sh, total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// Single workgroup: exclusive scan of the tile totals; writes the grand total
// to *total_out.  Each thread takes a contiguous run of the totals, so there
// is one workgroup scan whatever their number.
__global__ __launch_bounds__(BLOCK) void k_scan_top(int32_t *__restrict__ part, int ntiles, int32_t *total_out) {
  __shared__ int sh[BLOCK / 64];
  const int per = (ntiles + BLOCK - 1) / BLOCK;
  const int i0 = min((int)threadIdx.x * per, ntiles), i1 = min(i0 + per, ntiles);
  int sum = 0;
#pragma unroll 16
  for (int i = i0; i < i1; ++i) sum += part[i];
  int total;
  int run = block_excl_scan(sum, sh, total);
#pragma unroll 16
  for (int i = i0; i < i1; ++i) {
    const int v = part[i];
    part[i] = run;
    run += v;
  }
  if (threadIdx.x == 0) *total_out = total;
}

__global__ __launch_bounds__(BLOCK) void k_scan_apply(int32_t *__restrict__ in, long long n,
                                                      const int32_t *__restrict__ part, int32_t *__restrict__ out,
                                                      int zero_in) {
  __shared__ int sh[BLOCK / 64];
  const long long base = (long long)blockIdx.x * SCAN_TILE + (long long)threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  const bool full = scan_load8(in, base, n, v);
  int sum = 0;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; ++j) sum += v[j];
  int total;
  int run = part[blockIdx.x] + block_excl_scan(sum, sh, total);
  int o[SCAN_ITEMS];
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; ++j) {
    o[j] = run;
    run += v[j];
  }
  if (full) {
    *(int4 *)(out + base) = make_int4(o[0], o[1], o[2], o[3]);
    *(int4 *)(out + base + 4) = make_int4(o[4], o[5], o[6], o[7]);
    if (zero_in) {
      *(int4 *)(in + base) = make_int4(0, 0, 0, 0);
      *(int4 *)(in + base + 4) = make_int4(0, 0, 0, 0);
    }
  } else {
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j)
      if (base + j < n) {
        out[base + j] = o[j];
        if (zero_in) in[base + j] = 0;
      }
  }
}

// ------------------------------------------------------------------ particles per cell histogram
// hist[b] (b < nbins - 1): cells holding exactly b particles; hist[nbins - 1]:
// cells holding nbins - 1 or more, from the cell starts.  Counted per
// workgroup in LDS, then added to hist (cleared by the caller).
constexpr int HIST_BINS_MAX = 256;
__global__ __launch_bounds__(BLOCK) void k_count_hist(const int32_t *__restrict__ cs, int C, int nbins,
                                                      unsigned long long *hist) {
  __shared__ unsigned int h[HIST_BINS_MAX];
  for (int b = threadIdx.x; b < nbins; b += BLOCK) h[b] = 0;
  __syncthreads();
  for (int c = blockIdx.x * BLOCK + threadIdx.x; c < C; c += gridDim.x * BLOCK)
    atomicAdd(&h[min(cs[c + 1] - cs[c], nbins - 1)], 1u);
  __syncthreads();
  for (int b = threadIdx.x; b < nbins; b += BLOCK)
    if (h[b]) atomicAdd(&hist[b], (unsigned long long)h[b]);
}

// ------------------------------------------------------------------ FP64 conservation sums (fixed-order reductions)
__device__ __forceinline__ double block_sum_d(double v, double *sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < BLOCK / 64; ++w) t += sh[w];
  __syncthreads();
  return t;
}

template <int P>
__global__ __launch_bounds__(BLOCK) void k_cons_cells(const typename Prec<P>::S *__restrict__ f, int C,
                                                      double *__restrict__ part, int32_t *nonfinite) {
  __shared__ double sh[BLOCK / 64];
  double m = 0.0, px = 0.0, py = 0.0;
  int bad = 0;
  for (int c = blockIdx.x * BLOCK + threadIdx.x; c < C; c += gridDim.x * BLOCK) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double v = to_f64<P>(f, (size_t)i * C + c, i);
      bad |= !isfinite(v);
      m += v;
      px += (double)cx_of(i) * v;
      py += (double)cy_of(i) * v;
    }
  }
  if (bad) atomicOr(nonfinite, 1);
  const double a = block_sum_d(m, sh), b = block_sum_d(px, sh), c2 = block_sum_d(py, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x * 3 + 0] = a;
    part[blockIdx.x * 3 + 1] = b;
    part[blockIdx.x * 3 + 2] = c2;
  }
}

template <class T>
__global__ __launch_bounds__(BLOCK) void k_cons_parts(const T *__restrict__ vx, const T *__restrict__ vy, int n,
                                                      double mass, double *__restrict__ part, int32_t *nonfinite) {
  __shared__ double sh[BLOCK / 64];
  double qx = 0.0, qy = 0.0;
  int bad = 0;
  for (int s = blockIdx.x * BLOCK + threadIdx.x; s < n; s += gridDim.x * BLOCK) {
    const double a = (double)vx[s], b = (double)vy[s];
    bad |= !isfinite(a) || !isfinite(b);
    qx += mass * a;
    qy += mass * b;
  }
  if (bad) atomicOr(nonfinite, 1);
  const double a = block_sum_d(qx, sh), b = block_sum_d(qy, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x * 2 + 0] = a;
    part[blockIdx.x * 2 + 1] = b;
  }
}

__global__ __launch_bounds__(BLOCK) void k_cons_final(const double *__restrict__ pc, int nbc,
                                                      const double *__restrict__ pp, int nbp, const int32_t *nonfinite,
                                                      double *out) {
  __shared__ double sh[BLOCK / 64];
  double v[5] = {0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nbc; b += BLOCK)
    for (int j = 0; j < 3; ++j) v[j] += pc[b * 3 + j];
  for (int b = threadIdx.x; b < nbp; b += BLOCK)
    for (int j = 0; j < 2; ++j) v[3 + j] += pp[b * 2 + j];
  for (int j = 0; j < 5; ++j) {
    const double t = block_sum_d(v[j], sh);
    if (threadIdx.x == 0) out[j] = t;
  }
  if (threadIdx.x == 0) out[5] = *nonfinite ? 1.0 : 0.0;
}

// ------------------------------------------------------------------ layout conversion (canonical FP64 <-> internal)
template <int P>
__global__ __launch_bounds__(BLOCK) void k_set_f(const double *__restrict__ fin, typename Prec<P>::S *__restrict__ f,
                                                 int C) {
  const long long e = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (e >= (long long)Q * C) return;
  const int i = (int)(e / C);
  from_f64<P>(f, (size_t)e, i, fin ? fin[e] : wgt<double>(i));
}

template <int P>
__global__ __launch_bounds__(BLOCK) void k_get_f(const typename Prec<P>::S *__restrict__ f, double *__restrict__ out,
                                                 int C) {
  const long long e = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (e >= (long long)Q * C) return;
  out[e] = to_f64<P>(f, (size_t)e, (int)(e / C));
}

template <int P>
__global__ __launch_bounds__(BLOCK) void k_set_parts(const double *__restrict__ pos, const double *__restrict__ vel,
                                                     int n, Parts<typename Prec<P>::T> pt, int32_t *__restrict__ slot,
                                                     Consts<typename Prec<P>::T> k, int32_t *flags) {
  using T = typename Prec<P>::T;
  const int s = blockIdx.x * BLOCK + threadIdx.x;
  if (s >= n) return;
  double X = pos[2 * s], Y = pos[2 * s + 1];
  double fx = floor(X), fy = floor(Y);
  if (!(fx >= 0.0 && fx < k.nx && fy >= 0.0 && fy < k.ny)) {
    atomicOr(&flags[FLAG_DOMAIN], 1);
    X = 0.5;
    Y = 0.5;
    fx = 0.0;
    fy = 0.0;
  }
  int cx = (int)fx, cy = (int)fy;
  if constexpr (Prec<P>::global_pos) {
    pt.px[s] = (T)X;
    pt.py[s] = (T)Y;
  } else {
    T ox = (T)(X - fx), oy = (T)(Y - fy);
    if (ox >= (T)1) {  // rounding of the offset reached 1: carry
      ox = (T)0;
      cx += 1;
      if (cx >= k.nx) {
        if (k.per_x) cx = 0;
        else {
          cx = k.nx - 1;
          ox = (T)0.99999994f;
        }
      }
    }
    if (oy >= (T)1) {
      oy = (T)0;
      cy += 1;
      if (cy >= k.ny) {
        if (k.per_y) cy = 0;
        else {
          cy = k.ny - 1;
          oy = (T)0.99999994f;
        }
      }
    }
    pt.px[s] = ox;
    pt.py[s] = oy;
  }
  pt.key[s] = cy * k.nx + cx;
  pt.pid[s] = s;
  pt.vx[s] = (T)vel[2 * s];
  pt.vy[s] = (T)vel[2 * s + 1];
  slot[s] = s;
}

template <int P>
__global__ __launch_bounds__(BLOCK) void k_get_parts(Parts<typename Prec<P>::T> pt, const int32_t *__restrict__ slot,
                                                     int n, Consts<typename Prec<P>::T> k, double *pos, double *vel,
                                                     int32_t *cell, const typename Prec<P>::T *fdx,
                                                     const typename Prec<P>::T *fdy, double *fd) {
  const int g = blockIdx.x * BLOCK + threadIdx.x;
  if (g >= n) return;
  const int s = slot[g];
  const int key = pt.key[s];
  if (pos) {
    pos[2 * g] = Pos<P>::gx(k, key, pt.px[s]);
    pos[2 * g + 1] = Pos<P>::gy(k, key, pt.py[s]);
  }
  if (vel) {
    vel[2 * g] = (double)pt.vx[s];
    vel[2 * g + 1] = (double)pt.vy[s];
  }
  if (cell) {
    int cx, cy;
    cell_xy(k, key, cx, cy);
    cell[2 * g] = cx;
    cell[2 * g + 1] = cy;
  }
  if (fd) {
    fd[2 * g] = (double)fdx[g];
    fd[2 * g + 1] = (double)fdy[g];
  }
}

template <class T>
__global__ __launch_bounds__(BLOCK) void k_get_field(const T *__restrict__ a, const T *__restrict__ b, int C,
                                                     double *out, double add) {
  const int c = blockIdx.x * BLOCK + threadIdx.x;
  if (c >= C) return;
  if (b) {
    out[2 * c] = (double)a[c];
    out[2 * c + 1] = (double)b[c];
  } else {
    out[c] = add + (double)a[c];
  }
}

// Forward contacts (higher index) per particle index, then the pair list.
__global__ __launch_bounds__(BLOCK) void k_pairs_count(const int32_t *__restrict__ slot,
                                                       Adj adj,
                                                       const int32_t *__restrict__ deg, int n, int32_t *cnt) {
  const int g = blockIdx.x * BLOCK + threadIdx.x;
  if (g >= n) return;
  const int s = slot[g];
  const AdjRow row = adj.row(s);
  int c = 0;
  for (int a = 0; a < deg[s]; ++a) c += (int)(row[a] >> 32) > g;
  cnt[g] = c;
}

__global__ __launch_bounds__(BLOCK) void k_pairs_write(const int32_t *__restrict__ slot,
                                                       Adj adj,
                                                       const int32_t *__restrict__ deg, int n,
                                                       const int32_t *__restrict__ off, int32_t *pairs, long long cap) {
  const int g = blockIdx.x * BLOCK + threadIdx.x;
  if (g >= n) return;
  const int s = slot[g];
  const AdjRow row = adj.row(s);
  long long o = off[g];
  for (int a = 0; a < deg[s]; ++a) {
    const int j = (int)(row[a] >> 32);
    if (j > g) {
      if (o < cap) {
        pairs[2 * o] = g;
        pairs[2 * o + 1] = j;
      }
      ++o;
    }
  }
}

// ------------------------------------------------------------------ voidage statistics (Sec. 3 observables)
// The gas voidage of a cell is the 3-D voidage of Eq. 11 for its particle
// count, from an FP64 column of the per-count table.  Workgroups 0 .. ny-1 sum
// one row each (strided, then a fixed tree); the next ones take BLOCK columns
// each and walk rows y0 .. y1-1 in order, summing eps_g and counting the
// cells above the threshold (one partial count per workgroup).
__global__ __launch_bounds__(BLOCK) void k_voidage(const int32_t *__restrict__ cs, int nx, int ny, int nlut,
                                                   const double *__restrict__ eg_tab, int y0, int y1, double thr,
                                                   double *row_sum, double *col_sum, long long *part) {
  __shared__ double shd[BLOCK / 64];
  __shared__ long long shl[BLOCK / 64];
  const int b = blockIdx.x;
  if (b < ny) {
    if (!row_sum) return;
    double v = 0.0;
    for (int x = threadIdx.x; x < nx; x += BLOCK) {
      const int c = b * nx + x;
      v += eg_tab[min(cs[c + 1] - cs[c], nlut - 1)];
    }
    const double t = block_sum_d(v, shd);
    if (threadIdx.x == 0) row_sum[b] += t;
    return;
  }
  const int x = (b - ny) * BLOCK + (int)threadIdx.x;
  double v = 0.0;
  long long cnt = 0;
  if (x < nx) {
    for (int y = y0; y < y1; ++y) {
      const int c = y * nx + x;
      const double e = eg_tab[min(cs[c + 1] - cs[c], nlut - 1)];
      v += e;
      cnt += e > thr;
    }
    if (col_sum) col_sum[x] += v;
  }
  const long long t = block_sum_ll(cnt, shl);
  if (threadIdx.x == 0) part[b - ny] = t;
}

// One workgroup: the partial counts of k_voidage in a fixed order.
__global__ __launch_bounds__(BLOCK) void k_voidage_count(const long long *__restrict__ part, int n,
                                                         long long *out) {
  __shared__ long long shl[BLOCK / 64];
  long long v = 0;
  for (int i = threadIdx.x; i < n; i += BLOCK) v += part[i];
  const long long t = block_sum_ll(v, shl);
  if (threadIdx.x == 0) *out = t;
}

// The periodic check: a non-finite value found by the conservation sums
// (out[5] != 0) is latched in the context's flags.
__global__ void k_flag_nonfinite(const double *__restrict__ out, int32_t *flags) {
  if (threadIdx.x == 0 && out[5] != 0.0) atomicOr(&flags[FLAG_NONFINITE], 1);
}

__global__ void k_fill_i32(int32_t *p, long long n, int32_t v) {
  const long long i = (long long)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace lbdps
