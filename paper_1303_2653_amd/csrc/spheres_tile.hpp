// Hard-sphere stage of one tile of cells in LDS: contact detection (Sec. 2.2)
// and the binary collisions of Eqs. 17-18 for every contact cluster that lies
// inside the tile, with no neighbour rows written to memory.
//
// A workgroup loads the particles of a TW x TH tile of cells and of the ring of
// cells around it (positions of all; index and velocity of the tile's own), finds
// the contacts of the tile's particles with the same test as k_contacts, and
// joins them into clusters with a union-find over the contacts between the
// tile's particles.  A cluster with no contact into the ring, with at most
// ST_CMAX members and at most ST_KL contacts per member, is a whole cluster of
// the bed: every contact of its members was seen, and none leaves the tile.
// One lane resolves it as the cluster kernel does (members in index order, each
// meeting its higher-index neighbours in index order, then its wall pass), so
// the result is the sequential sweep's bit for bit.  A particle with no
// contact takes its wall pass here.  The tile marks every particle it resolved
// (done = DONE_WHOLE) and leaves the others (done = 0) to the row-based path:
// k_contacts in its skipping form, the cluster kernel and the ordered sweep.
// A cluster is either resolved here whole or left whole: a cluster that
// crosses the tile's edge has, in the tile, only parts that each touch the ring.
#pragma once

#include "kernels.hpp"

namespace lbdps {

constexpr int ST_KL = 6;     // contacts kept per particle in LDS
constexpr int ST_CMAX = 64;  // most members of a cluster one lane resolves
constexpr int ST_ITER = 48;  // union-find rounds before the tile leaves its clusters to the row path

template <int TW, int TH> struct StShape {
  static constexpr int LW = TW + 2, LH = TH + 2, NLC = LW * LH;   // the tile and its ring
  static constexpr int MAXP = ((NLC * 5 / 3) + 63) / 64 * 64;       // particles held
  static constexpr int CPT = (NLC + BLOCK - 1) / BLOCK;             // cells per thread
};

template <class T, int TW, int TH> struct StLds {
  using S = StShape<TW, TH>;
  T x[S::MAXP], y[S::MAXP], vx[S::MAXP], vy[S::MAXP];
  int pid[S::MAXP];
  int par[S::MAXP];  // union-find parent (a lower local index); the root after compression
  int csz[S::MAXP];  // cluster size, at the root
  int cur[S::MAXP];  // next member place, at the root
  unsigned short cell[S::MAXP];
  unsigned short mem[S::MAXP];  // members grouped by cluster
  unsigned short ct[ST_KL][S::MAXP];
  unsigned char nc[S::MAXP];
  unsigned char open[S::MAXP];   // the particle has a contact in the ring or more than ST_KL
  unsigned char copen[S::MAXP];  // at a root: some member is open
  unsigned char dirty[S::MAXP];  // velocity changed
  int lstart[S::NLC + 1];        // first local particle of each local cell
  int gstart[S::NLC];            // slot of the cell's first particle
  int gkey[S::NLC];              // cell key (-1: beyond a wall)
  int stamp, cursor;
};

// Tile shapes (the tuning field sphere_tile): 0 = no tile kernel, every
// particle through the row path; 1 = 32 x 8 cells; 2 = 16 x 16; 3 = 64 x 4.
constexpr int SPHERE_TILES = 4;
__host__ __device__ constexpr void sphere_tile_dims(int t, int &tw, int &th) {
  tw = t == 2 ? 16 : (t == 3 ? 64 : 32);
  th = t == 2 ? 16 : (t == 3 ? 4 : 8);
}

// Tiles of a bed for the tile shape (TW, TH).
__host__ __device__ constexpr int st_tiles(int nx, int ny, int tw, int th) {
  return ((nx + tw - 1) / tw) * ((ny + th - 1) / th);
}

template <int P, int TW, int TH>
__device__ __forceinline__ void spheres_tile_body(const int bidx, Parts<typename Prec<P>::T> pt,
    const int32_t *__restrict__ cs, const Consts<typename Prec<P>::T> &k, int32_t *__restrict__ done,
    long long *__restrict__ tpart, const int ntiles) {
  using T = typename Prec<P>::T;
  using S = StShape<TW, TH>;
  __shared__ StLds<T, TW, TH> L;
  __shared__ int shi[BLOCK / 64];
  __shared__ long long sh[BLOCK / 64];
  const int tid = threadIdx.x;
  const int ntx = (k.nx + TW - 1) / TW;
  const int x0 = (bidx % ntx) * TW, y0 = (bidx / ntx) * TH;
  const int w = min(TW, k.nx - x0), h = min(TH, k.ny - y0);  // the tile, clipped to the bed
  auto inside = [&](int lc) {
    const int lx = lc % S::LW, ly = lc / S::LW;
    return lx >= 1 && lx <= w && ly >= 1 && ly <= h;
  };
  // 1. cells of the tile and its ring (wrapped across periodic faces, empty
  // beyond walls and beyond the clipped tile), and their particle counts
  int cnt[S::CPT];
  int mine = 0;
#pragma unroll
  for (int j = 0; j < S::CPT; ++j) {
    const int lc = tid * S::CPT + j;
    int c = 0;
    if (lc < S::NLC) {
      const int lx = lc % S::LW, ly = lc / S::LW;
      int g = -1, a = 0;
      if (lx <= w + 1 && ly <= h + 1) {
        int gx = x0 + lx - 1, gy = y0 + ly - 1;
        bool ok = true;
        if (gx < 0 || gx >= k.nx) {
          ok = k.per_x != 0;
          gx = wrap_i(gx, k.nx);
        }
        if (gy < 0 || gy >= k.ny) {
          ok = ok && k.per_y != 0;
          gy = wrap_i(gy, k.ny);
        }
        if (ok) {
          g = gy * k.nx + gx;
          a = cs[g];
          c = cs[g + 1] - a;
        }
      }
      L.gstart[lc] = a;
      L.gkey[lc] = g;
    }
    cnt[j] = c;
    mine += c;
  }
  int M;
  int off = block_excl_scan(mine, shi, M);
#pragma unroll
  for (int j = 0; j < S::CPT; ++j) {
    const int lc = tid * S::CPT + j;
    if (lc < S::NLC) L.lstart[lc] = off;
    off += cnt[j];
  }
  if (tid == 0) {
    L.lstart[S::NLC] = M;
    L.stamp = 0;
    L.cursor = 0;
  }
  long long npair = 0, ncoll = 0, nwall = 0;
  bool whole = M <= S::MAXP;  // uniform
  __syncthreads();
  if (whole) {
    // 2. the particles, in cell order
    for (int q = tid; q < M; q += BLOCK) {
      int lo = 0, hi = S::NLC;  // lstart[lo] <= q < lstart[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (L.lstart[mid] <= q) lo = mid;
        else hi = mid;
      }
      const int s = L.gstart[lo] + (q - L.lstart[lo]);
      L.cell[q] = (unsigned short)lo;
      L.x[q] = pt.px[s];
      L.y[q] = pt.py[s];
      L.par[q] = q;
      L.csz[q] = 0;
      L.nc[q] = 0;
      L.open[q] = 0;
      L.copen[q] = 0;
      L.dirty[q] = 0;
      if (inside(lo)) {
        L.pid[q] = pt.pid[s];
        L.vx[q] = pt.vx[s];
        L.vy[q] = pt.vy[s];
      }
    }
    __syncthreads();
    // 3. contacts of the tile's particles: the particle's cell and its eight
    // neighbours, the distance test of k_contacts
    const T dd = k.d * k.d;
    for (int q = tid; q < M; q += BLOCK) {
      const int lc = L.cell[q];
      if (!inside(lc)) continue;
      const T x = L.x[q], y = L.y[q];
      int n = 0;
      bool op = false;
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
          const int nb = lc + oy * S::LW + ox;
          const int t1 = L.lstart[nb + 1];
          for (int t = L.lstart[nb]; t < t1; ++t) {
            if (t == q) continue;
            T dx, dy;
            Pos<P>::sep_nb(k, ox, oy, x, y, L.x[t], L.y[t], dx, dy);
            if (dx * dx + dy * dy <= dd) {
              if (!inside(L.cell[t]) || n == ST_KL) {
                op = true;
              } else {
                L.ct[n][q] = (unsigned short)t;
                ++n;
              }
            }
          }
        }
      L.nc[q] = (unsigned char)n;
      L.open[q] = op ? 1 : 0;
    }
    __syncthreads();
    // 4. clusters: union-find over the kept contacts (both directions, so a
    // contact kept by one side only still joins), then path compression
    auto find = [&](int a) {
      while (L.par[a] != a) a = L.par[a];
      return a;
    };
    for (int it = 1;; ++it) {
      for (int q = tid; q < M; q += BLOCK) {
        const int n = L.nc[q];
        for (int a = 0; a < n; ++a) {
          const int r1 = find(q), r2 = find(L.ct[a][q]);
          if (r1 != r2) {
            atomicMin(&L.par[max(r1, r2)], min(r1, r2));
            L.stamp = it;
          }
        }
      }
      __syncthreads();
      for (int q = tid; q < M; q += BLOCK) L.par[q] = find(q);
      const bool again = L.stamp == it;  // written before the barrier above, next written after the one below
      __syncthreads();
      if (!again) break;
      if (it == ST_ITER) {  // uniform: leave every cluster of the tile to the row path
        whole = false;
        break;
      }
    }
  }
  if (whole) {
    // 5. cluster sizes and open clusters
    for (int q = tid; q < M; q += BLOCK) {
      if (!inside(L.cell[q])) continue;
      const int r = L.par[q];
      atomicAdd(&L.csz[r], 1);
      if (L.open[q]) L.copen[r] = 1;
    }
    __syncthreads();
    auto resolvable = [&](int r) { return !L.copen[r] && L.csz[r] <= ST_CMAX; };
    // 6. member lists of the clusters resolved here
    for (int q = tid; q < M; q += BLOCK)
      if (L.par[q] == q && inside(L.cell[q]) && L.csz[q] >= 2 && resolvable(q))
        L.cur[q] = atomicAdd(&L.cursor, L.csz[q]);
    __syncthreads();
    for (int q = tid; q < M; q += BLOCK) {
      if (!inside(L.cell[q])) continue;
      const int r = L.par[q];
      if (L.csz[r] >= 2 && resolvable(r)) L.mem[atomicAdd(&L.cur[r], 1)] = (unsigned short)q;
    }
    __syncthreads();
    // 7. one lane per cluster: members by index, each with its higher-index
    // neighbours by index, then its wall pass; a particle without contacts
    // takes its wall pass alone
    for (int q = tid; q < M; q += BLOCK) {
      if (!inside(L.cell[q]) || L.par[q] != q || !resolvable(q)) continue;
      const int m = L.csz[q];
      if (m == 1) {
        T vx = L.vx[q], vy = L.vy[q];
        const int hw = Pos<P>::walls_key(k, L.gkey[L.cell[q]], L.x[q], L.y[q], vx, vy);
        if (hw) {
          L.vx[q] = vx;
          L.vy[q] = vy;
          L.dirty[q] = 1;
          nwall += hw;
        }
        continue;
      }
      const int base = L.cur[q] - m;
      for (int i = 1; i < m; ++i) {
        const int e = L.mem[base + i], pe = L.pid[e];
        int j = i - 1;
        while (j >= 0 && L.pid[L.mem[base + j]] > pe) {
          L.mem[base + j + 1] = L.mem[base + j];
          --j;
        }
        L.mem[base + j + 1] = (unsigned short)e;
      }
      for (int i = 0; i < m; ++i) {
        const int u = L.mem[base + i];
        const int pu = L.pid[u], ku = L.gkey[L.cell[u]], nu = L.nc[u];
        const T xu = L.x[u], yu = L.y[u];
        T vxu = L.vx[u], vyu = L.vy[u];
        bool du = false;
        for (int last = pu;;) {  // the next higher neighbour by index
          int wb = -1, pb = 0;
          for (int a = 0; a < nu; ++a) {
            const int t = L.ct[a][u], p = L.pid[t];
            if (p > last && (wb < 0 || p < pb)) {
              wb = t;
              pb = p;
            }
          }
          if (wb < 0) break;
          last = pb;
          ++npair;
          T dx, dy;
          Pos<P>::sep(k, ku, xu, yu, L.gkey[L.cell[wb]], L.x[wb], L.y[wb], dx, dy);
          T vxw = L.vx[wb], vyw = L.vy[wb];
          if (pair_core<P>(k, dx, dy, vxu, vyu, vxw, vyw)) {
            L.vx[wb] = vxw;
            L.vy[wb] = vyw;
            L.dirty[wb] = 1;
            du = true;
            ++ncoll;
          }
        }
        const int hw = Pos<P>::walls_key(k, ku, xu, yu, vxu, vyu);
        nwall += hw;
        if (du || hw) {
          L.vx[u] = vxu;
          L.vy[u] = vyu;
          L.dirty[u] = 1;
        }
      }
    }
    __syncthreads();
    // 8. marks and changed velocities of the tile's particles
    for (int q = tid; q < M; q += BLOCK) {
      const int lc = L.cell[q];
      if (!inside(lc)) continue;
      const int s = L.gstart[lc] + (q - L.lstart[lc]);
      const bool res = resolvable(L.par[q]);
      done[s] = res ? DONE_WHOLE : 0;
      if (res && L.dirty[q]) {
        pt.vx[s] = L.vx[q];
        pt.vy[s] = L.vy[q];
      }
    }
  } else {
    // the tile holds more particles than LDS, or its clusters did not settle:
    // all of its particles go to the row path
    for (int r = 0; r < h; ++r) {
      const int g0 = (y0 + r) * k.nx + x0;
      const int a = cs[g0], b = cs[g0 + w];
      for (int s = a + tid; s < b; s += BLOCK) done[s] = 0;
    }
  }
  const long long tp = block_sum_ll(npair, sh);
  const long long tc = block_sum_ll(ncoll, sh);
  const long long tw = block_sum_ll(nwall, sh);
  if (tid == 0) {
    tpart[bidx] = tp;
    tpart[ntiles + bidx] = tc;
    tpart[2 * ntiles + bidx] = tw;
  }
}

template <int P, int TW, int TH>
__global__ __launch_bounds__(BLOCK) void k_spheres_tile(Parts<typename Prec<P>::T> pt, const int32_t *__restrict__ cs,
                                                        Consts<typename Prec<P>::T> k, int32_t *__restrict__ done,
                                                        long long *__restrict__ tpart) {
  spheres_tile_body<P, TW, TH>(xcd_block<XCD_RUN_CONTACTS>(blockIdx.x, gridDim.x), pt, cs, k, done, tpart,
                               (int)gridDim.x);
}

}  // namespace lbdps
