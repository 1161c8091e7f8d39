// Hard-sphere stage of one tile of cells in LDS: contact detection (Sec. 2.2)
// and the binary collisions of Eqs. 17-18, with neighbour rows written only
// for the few particles whose cluster no tile can resolve.
//
// A workgroup loads the particles of a TW x TH tile of cells and of two rings
// of cells around it.  The tile and the inner ring form its inner region: the
// contacts of every particle there are all among the loaded particles.  It
// finds those contacts with the contact kernel's test, and each particle of
// the inner region whose contacts all have higher indices (a candidate root)
// gathers its cluster breadth-first into a queue of its own, giving up at a
// lower index.  A gathered cluster is resolvable when
//   - no member has a contact outside the inner region or more than ST_KL,
//   - it has at most ST_CM members, and
//   - it lies in the inner region of the tile of each of its members (a
//     cluster reaching into a neighbouring tile's first row or column of
//     cells, and no further, qualifies).
// and no member's tile holds more particles (with its rings) than its LDS
// takes.  Every tile holding a member sees the same cluster and reaches the
// same verdict (each counts what its neighbours hold from the cell starts), so
// each tile marks its own members resolved or not without talking to the
// others.  The tile holding the cluster's lowest index
// resolves it on one lane: members in index order, each meeting its
// higher-index neighbours in index order, then its wall pass, as the cluster
// kernel does, so the result is the sequential sweep's bit for bit.  A
// particle without contacts takes its wall pass in its tile.  For a particle
// whose cluster is not resolvable the tile writes what the contact kernel
// would: its sorted neighbour row, its degree, the chunk mark, and, for a
// candidate root, an entry in one compact list that the cluster kernel and
// the ordered sweep then take as before.
//
// Along a periodic axis shorter than the tile and its rings, the rings hold
// copies of the tile's own cells; there the inner region is the tile itself.
#pragma once

#include "kernels.hpp"

namespace lbdps {

constexpr int ST_H = 2;    // rings of cells around the tile
constexpr int ST_KL = 6;   // contacts kept per particle in LDS
constexpr int ST_CM = 16;  // most members of a cluster a tile resolves
constexpr int ST_CH = 4;   // contact candidates loaded together
constexpr int ST_ITER = 20;  // label rounds (at least ST_CM - 1)
static_assert(ST_ITER >= ST_CM - 1, "a cluster the tile may resolve is labelled within the rounds");

template <int TW, int TH> struct StShape {
  static constexpr int LW = TW + 2 * ST_H, LH = TH + 2 * ST_H, NLC = LW * LH;  // the tile and its rings
  static constexpr int MAXP = ((NLC * 5 / 3) + 63) / 64 * 64;                   // particles held
  static constexpr int CPT = (NLC + BLOCK - 1) / BLOCK;                         // cells per thread
};

template <class T, int TW, int TH> struct StLds {
  using S = StShape<TW, TH>;
  T x[S::MAXP], y[S::MAXP], vx[S::MAXP], vy[S::MAXP];
  int pid[S::MAXP];
  unsigned short cell[S::MAXP];
  unsigned short ct[ST_KL][S::MAXP];  // contacts in the inner region (local indices)
  unsigned char nc[S::MAXP];          // contacts kept
  unsigned char ntot[S::MAXP];        // all contacts (up to 255)
  unsigned char open[S::MAXP];        // a contact outside the inner region, or more than ST_KL
  unsigned char res[S::MAXP];         // a tile's particle whose cluster is resolved
  unsigned short lab[S::MAXP];        // cluster label: the lowest-index member found so far
  unsigned short mem[S::MAXP];        // members of the clusters this tile resolves
  unsigned short sorted[S::MAXP];     // the same, each cluster's members in index order
  int agg[S::MAXP];                   // at a root: member count << 16 | verdict marks
  int cur[S::MAXP];                   // at a root: the cluster's first place in mem / sorted
  int cur2[S::MAXP];                  // at a root: members placed so far
  int cursor;
  int lstart[S::NLC + 1];             // first local particle of each local cell
  int gstart[S::NLC];                 // slot of the cell's first particle
  int held[9];                        // particles the 3 x 3 tiles around this one (row-major) would hold
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

// The row path's inputs for slot s, from global memory (for a tile beyond the
// LDS capacity): the contacts over the 3 x 3 cells with the contact kernel's
// test, the sorted row, degree, mark, chunk mark and compact root entry; a
// particle without contacts takes its wall pass.
template <int P>
__device__ void st_row_global(Parts<typename Prec<P>::T> pt, const int32_t *__restrict__ cs,
                              const Consts<typename Prec<P>::T> &k, Adj adj, int32_t *__restrict__ deg,
                              int32_t *__restrict__ done, int32_t *__restrict__ chunk_busy, long long *__restrict__ roots,
                              int32_t *nroots, const int s, long long &npair, long long &nwall) {
  using T = typename Prec<P>::T;
  const int id = pt.pid[s];
  int cx, cy;
  cell_xy(k, pt.key[s], cx, cy);
  const T x = pt.px[s], y = pt.py[s], dd = k.d * k.d;
  const AdjRow row = adj.row(s);
  int cnt = 0, lowest = 0x7fffffff;
  bool over = false;
  for (int oy = -1; oy <= 1; ++oy) {
    int yy = cy + oy;
    if (yy < 0 || yy >= k.ny) {
      if (!k.per_y) continue;
      yy = wrap_i(yy, k.ny);
    }
    for (int ox = -1; ox <= 1; ++ox) {
      int xx = cx + ox;
      if (xx < 0 || xx >= k.nx) {
        if (!k.per_x) continue;
        xx = wrap_i(xx, k.nx);
      }
      const int c = yy * k.nx + xx;
      for (int t = cs[c]; t < cs[c + 1]; ++t) {
        if (t == s) continue;
        T dx, dy;
        Pos<P>::sep_nb(k, ox, oy, x, y, pt.px[t], pt.py[t], dx, dy);
        if (!(dx * dx + dy * dy <= dd)) continue;
        const int tid = pt.pid[t];
        npair += tid > id;
        lowest = min(lowest, tid);
        if (cnt == KMAX) {
          over = true;
          continue;
        }
        const long long e = ((long long)tid << 32) | (unsigned)t;
        int j = cnt;
        while (j > 0 && row[j - 1] > e) {
          row[j] = row[j - 1];
          --j;
        }
        row[j] = e;
        ++cnt;
      }
    }
  }
  if (cnt == 0) {
    T vx = pt.vx[s], vy = pt.vy[s];
    const int hw = Pos<P>::walls(k, cx, cy, x, y, vx, vy);
    if (hw) {
      pt.vx[s] = vx;
      pt.vy[s] = vy;
      nwall += hw;
    }
    done[s] = DONE_WHOLE;
    return;
  }
  if (over) atomicOr(&k.flags[FLAG_CAPACITY], 1);
  deg[s] = cnt;
  done[s] = 0;
  chunk_busy[id / RES_CHUNK] = 1;
  if (lowest > id) roots[atomicAdd(nroots, 1)] = ((long long)id << 32) | (unsigned)s;
}

// tpart: per tile, [4][ntiles]: contact pairs, collisions and wall hits of the
// particles it resolved, and the particles it left to the row path.
// nroots: the compact list's length (zeroed by the ordered sweep kernel at the
// end of every collision stage); roots: the list.
template <int P, int TW, int TH>
__device__ __forceinline__ void spheres_tile_body(const int bidx, Parts<typename Prec<P>::T> pt,
    const int32_t *__restrict__ cs, const Consts<typename Prec<P>::T> &k, Adj adj, int32_t *__restrict__ deg,
    int32_t *__restrict__ done, int32_t *ticket, int32_t *need_sweep, int32_t *__restrict__ chunk_busy,
    long long *__restrict__ roots, long long *__restrict__ tpart, const int ntiles) {
  using T = typename Prec<P>::T;
  using S = StShape<TW, TH>;
  constexpr int H = ST_H;
  __shared__ StLds<T, TW, TH> L;
  __shared__ int shi[BLOCK / 64];
  __shared__ long long sh[BLOCK / 64];
  const int tid = threadIdx.x;
  if (bidx == 0 && tid == 0) {  // read only by the kernels after this one
    *ticket = 0;
    need_sweep[0] = 0;
  }
  const int ntx = (k.nx + TW - 1) / TW;
  const int x0 = (bidx % ntx) * TW, y0 = (bidx / ntx) * TH;
  const int w = min(TW, k.nx - x0), h = min(TH, k.ny - y0);  // the tile, clipped to the bed
  // rings that copy the tile's own cells (short periodic axes): inner region = tile
  const bool dupx = k.per_x && k.nx < TW + 2 * H, dupy = k.per_y && k.ny < TH + 2 * H;
  const int ix0 = dupx ? H : H - 1, ix1 = dupx ? w + H - 1 : w + H;
  const int iy0 = dupy ? H : H - 1, iy1 = dupy ? h + H - 1 : h + H;
  auto in_tile = [&](int lc) {
    const int lx = lc % S::LW, ly = lc / S::LW;
    return lx >= H && lx < w + H && ly >= H && ly < h + H;
  };
  auto in_inner = [&](int lc) {
    const int lx = lc % S::LW, ly = lc / S::LW;
    return lx >= ix0 && lx <= ix1 && ly >= iy0 && ly <= iy1;
  };
  auto slot_of = [&](int q) { return L.gstart[L.cell[q]] + (q - L.lstart[L.cell[q]]); };
  auto key_of = [&](int q) {
    const int lc = L.cell[q];
    const int gx = wrap_i(x0 + lc % S::LW - H, k.nx), gy = wrap_i(y0 + lc / S::LW - H, k.ny);
    return gy * k.nx + gx;
  };
  if (tid < 9) L.held[tid] = 0;
  // 1. cells of the tile and its rings (wrapped across periodic faces, empty
  // beyond walls and beyond the clipped tile's rings), their particle counts
  int cnt[S::CPT];
  int mine = 0;
#pragma unroll
  for (int j = 0; j < S::CPT; ++j) {
    const int lc = tid * S::CPT + j;
    int c = 0;
    if (lc < S::NLC) {
      const int lx = lc % S::LW, ly = lc / S::LW;
      int a = 0;
      if (lx < w + 2 * H && ly < h + 2 * H) {
        int gx = x0 + lx - H, gy = y0 + ly - H;
        bool ok = true;
        if (gx < 0 || gx >= k.nx) {
          ok = k.per_x != 0;
          gx = gx < 0 ? gx + k.nx : gx - k.nx;
        }
        if (gy < 0 || gy >= k.ny) {
          ok = ok && k.per_y != 0;
          gy = gy < 0 ? gy + k.ny : gy - k.ny;
        }
        if (ok) {
          const int g = gy * k.nx + gx;
          a = cs[g];
          c = cs[g + 1] - a;
        }
      }
      L.gstart[lc] = a;
    }
    cnt[j] = c;
    mine += c;
  }
  int M;
  int off = block_excl_scan(mine, shi, M);
#pragma unroll
  for (int j = 0; j < S::CPT; ++j) {
    const int lc = tid * S::CPT + j;
    if (lc < S::NLC) {
      L.lstart[lc] = off;
      for (int i = off; i < min(off + cnt[j], S::MAXP); ++i) L.cell[i] = (unsigned short)lc;
    }
    off += cnt[j];
  }
  if (tid == 0) {
    L.lstart[S::NLC] = M;
    L.cursor = 0;
  }
  // what the 3 x 3 tiles around this one hold with their rings, counted the way
  // each counts its own: per row of its rings, the runs of cells between
  // periodic seams (the tile itself: M)
  {
    const int tx = bidx % ntx, ty = bidx / ntx, nty = (k.ny + TH - 1) / TH;
    for (int i = tid; i < 9 * (TH + 2 * H); i += BLOCK) {
      const int n = i / (TH + 2 * H), r = i % (TH + 2 * H);
      int tnx = tx + n % 3 - 1, tny = ty + n / 3 - 1;
      if (tnx < 0 || tnx >= ntx) {
        if (!k.per_x) continue;
        tnx = tnx < 0 ? ntx - 1 : 0;
      }
      if (tny < 0 || tny >= nty) {
        if (!k.per_y) continue;
        tny = tny < 0 ? nty - 1 : 0;
      }
      const int xn = tnx * TW, wn = min(TW, k.nx - xn), yn = tny * TH, hn = min(TH, k.ny - yn);
      if (r >= hn + 2 * H) continue;
      int gy = yn - H + r;
      if (gy < 0 || gy >= k.ny) {
        if (!k.per_y) continue;
        gy = gy < 0 ? gy + k.ny : gy - k.ny;
      }
      const int a = xn - H, b = xn + wn + H - 1, base = gy * k.nx;
      int c = cs[base + min(b, k.nx - 1) + 1] - cs[base + max(a, 0)];
      if (k.per_x) {
        if (a < 0) c += cs[base + k.nx] - cs[base + a + k.nx];
        if (b >= k.nx) c += cs[base + b - k.nx + 1] - cs[base];
      }
      atomicAdd(&L.held[n], c);
    }
  }
  long long npair = 0, ncoll = 0, nwall = 0, nleft = 0;
  const bool whole = M <= S::MAXP;  // uniform
  __syncthreads();
  if (whole) {
    // 2. the particles, in cell order: positions and indices of all,
    // velocities of the inner region's
    for (int q = tid; q < M; q += BLOCK) {
      const int lo = L.cell[q];
      const int s = L.gstart[lo] + (q - L.lstart[lo]);
      L.x[q] = pt.px[s];
      L.y[q] = pt.py[s];
      L.pid[q] = pt.pid[s];
      L.res[q] = 0;
      if (in_inner(lo)) {
        L.vx[q] = pt.vx[s];
        L.vy[q] = pt.vy[s];
      }
    }
    __syncthreads();
    // 3. contacts of the inner region's particles: the cell and its eight
    // neighbours, the distance test of k_contacts.  The three cells of a row
    // are one run of local particles; the runs' bounds are read together and
    // the candidates ST_CH at a time, loads before tests.  The kept contacts
    // are sorted by particle index (in registers, then stored).
    const T dd = k.d * k.d;
    for (int q = tid; q < M; q += BLOCK) {
      const int lc = L.cell[q];
      if (!in_inner(lc)) continue;
      const T x = L.x[q], y = L.y[q];
      int rb[3][4];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int e = 0; e < 4; ++e) rb[r][e] = L.lstart[lc + (r - 1) * S::LW + e - 1];
      const int n0 = rb[0][3] - rb[0][0], n01 = n0 + rb[1][3] - rb[1][0], tot = n01 + rb[2][3] - rb[2][0];
      long long kept[ST_KL];  // (index << 16 | local index), ascending
      int n = 0, all = 0;
      bool op = false;
      for (int q0 = 0; q0 < tot; q0 += ST_CH) {
        int tt[ST_CH], ox[ST_CH], oy[ST_CH], ids[ST_CH];
        T xs[ST_CH], ys[ST_CH];
#pragma unroll
        for (int j = 0; j < ST_CH; ++j) {
          const int i = min(q0 + j, tot - 1);
          const int r = i < n0 ? 0 : (i < n01 ? 1 : 2);
          const int t = i - (r == 0 ? 0 : (r == 1 ? n0 : n01)) + (r == 0 ? rb[0][0] : (r == 1 ? rb[1][0] : rb[2][0]));
          const int b1 = r == 0 ? rb[0][1] : (r == 1 ? rb[1][1] : rb[2][1]);
          const int b2 = r == 0 ? rb[0][2] : (r == 1 ? rb[1][2] : rb[2][2]);
          tt[j] = t;
          ox[j] = t < b1 ? -1 : (t < b2 ? 0 : 1);
          oy[j] = r - 1;
          xs[j] = L.x[t];
          ys[j] = L.y[t];
          ids[j] = L.pid[t];
        }
#pragma unroll
        for (int j = 0; j < ST_CH; ++j) {
          if (q0 + j >= tot || tt[j] == q) continue;
          T dx, dy;
          Pos<P>::sep_nb(k, ox[j], oy[j], x, y, xs[j], ys[j], dx, dy);
          if (dx * dx + dy * dy <= dd) {
            ++all;
            if (!in_inner(lc + oy[j] * S::LW + ox[j]) || n == ST_KL) {
              op = true;
            } else {
              const long long e = ((long long)ids[j] << 16) | tt[j];
              bool placed = false;
#pragma unroll
              for (int u = ST_KL - 1; u >= 0; --u)
                if (!placed && u <= n) {
                  if (u > 0 && kept[u - 1] > e) {
                    kept[u] = kept[u - 1];
                  } else {
                    kept[u] = e;
                    placed = true;
                  }
                }
              ++n;
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < ST_KL; ++u)
        if (u < n) L.ct[u][q] = (unsigned short)(kept[u] & 0xffff);
      L.nc[q] = (unsigned char)n;
      L.ntot[q] = (unsigned char)min(all, 255);
      L.open[q] = op ? 1 : 0;
      L.lab[q] = (unsigned short)q;
      L.agg[q] = 0;
      L.cur2[q] = 0;
    }
    __syncthreads();
    // 4. clusters.  Each particle of the inner region takes the lowest-index
    // label among its contacts' until no label changes: the label is then the
    // cluster's lowest-index member, its root.  A cluster of m members is
    // labelled after m - 1 rounds; one still mixing labels after the last round
    // is larger than ST_CM and is caught below (a member whose contact carries
    // another label marks its group open).
    for (int it = 0; it < ST_ITER; ++it) {
      bool changed = false;
      for (int q = tid; q < M; q += BLOCK) {
        const int n = L.nc[q];
        if (n == 0 || !in_inner(L.cell[q])) continue;
        const int cur = L.lab[q];
        int best = cur, bp = L.pid[cur];
        for (int a = 0; a < n; ++a) {
          const int lt = L.lab[L.ct[a][q]], pl = L.pid[lt];
          if (pl < bp) {
            bp = pl;
            best = lt;
          }
        }
        if (best != cur) {
          L.lab[q] = (unsigned short)best;
          changed = true;
        }
      }
      if (!__syncthreads_or(changed)) break;
    }
    // per root: member count (high bits) and the marks of the verdict (low bits)
    constexpr int A_OPEN = 1, A_FULL = 2, A_XL = 4, A_XLI = 8, A_XR = 16, A_XRI = 32, A_YB = 64, A_YBI = 128,
                  A_YT = 256, A_YTI = 512, A_ONE = 1 << 16;
    for (int q = tid; q < M; q += BLOCK) {
      const int lc = L.cell[q];
      if (L.nc[q] == 0 || !in_inner(lc)) continue;
      const int lx = lc % S::LW, ly = lc / S::LW;
      const int ox = lx < H ? 0 : (lx >= w + H ? 2 : 1), oy = ly < H ? 0 : (ly >= h + H ? 2 : 1);
      const int lq = L.lab[q];
      bool mixed = false;
      for (int a = 0; a < L.nc[q]; ++a) mixed = mixed || L.lab[L.ct[a][q]] != lq;
      int f = A_ONE | (L.open[q] || mixed ? A_OPEN : 0) | (L.held[oy * 3 + ox] > S::MAXP ? A_FULL : 0);
      f |= (lx < H ? A_XL : 0) | (lx > H ? A_XLI : 0) | (lx >= w + H ? A_XR : 0) | (lx < w + H - 1 ? A_XRI : 0);
      f |= (ly < H ? A_YB : 0) | (ly > H ? A_YBI : 0) | (ly >= h + H ? A_YT : 0) | (ly < h + H - 1 ? A_YTI : 0);
      atomicAdd(&L.agg[lq], f & ~0xffff);
      atomicOr(&L.agg[lq], f & 0xffff);
    }
    __syncthreads();
    // The verdict (the same in every tile holding a member): no member open or
    // in a tile beyond its capacity, at most ST_CM members, and within the
    // inner region of each member's tile (a member in the left ring of cells
    // forbids members right of this tile's first column, and so on).
    auto resolvable = [&](int r) {
      const int f = L.agg[r];
      return (f >> 16) <= ST_CM && !(f & (A_OPEN | A_FULL)) && !((f & A_XL) && (f & A_XLI)) &&
             !((f & A_XR) && (f & A_XRI)) && !((f & A_YB) && (f & A_YBI)) && !((f & A_YT) && (f & A_YTI));
    };
    for (int q = tid; q < M; q += BLOCK) {
      const int lc = L.cell[q];
      if (L.nc[q] == 0 || !in_inner(lc)) continue;
      const int r = L.lab[q];
      const bool ok = resolvable(r);
      if (ok && in_tile(lc)) L.res[q] = 1;
      if (ok && r == q && in_tile(lc)) L.cur[q] = atomicAdd(&L.cursor, L.agg[q] >> 16);  // this tile resolves it
    }
    __syncthreads();
    // members of the clusters this tile resolves, then each member's place in
    // index order among them
    for (int q = tid; q < M; q += BLOCK) {
      const int lc = L.cell[q];
      if (L.nc[q] == 0 || !in_inner(lc)) continue;
      const int r = L.lab[q];
      if (in_tile(L.cell[r]) && resolvable(r)) L.mem[atomicAdd(&L.cur2[r], 1) + L.cur[r]] = (unsigned short)q;
    }
    __syncthreads();
    for (int q = tid; q < M; q += BLOCK) {
      const int lc = L.cell[q];
      if (L.nc[q] == 0 || !in_inner(lc)) continue;
      const int r = L.lab[q];
      if (!in_tile(L.cell[r]) || !resolvable(r)) continue;
      const int base = L.cur[r], m = L.agg[r] >> 16, pq = L.pid[q];
      int rank = 0;
      for (int i = 0; i < m; ++i) rank += L.pid[L.mem[base + i]] < pq;
      L.sorted[base + rank] = (unsigned short)q;
    }
    __syncthreads();
    // one lane per cluster: members in index order, each with its higher-index
    // neighbours in index order (its sorted contacts), then its wall pass
    for (int q = tid; q < M; q += BLOCK) {
      const int lc = L.cell[q];
      if (L.nc[q] == 0 || L.lab[q] != q || !in_tile(lc) || !resolvable(q)) continue;
      const int base = L.cur[q], m = L.agg[q] >> 16;
      for (int i = 0; i < m; ++i) {
        const int u = L.sorted[base + i];
        const int pu = L.pid[u], ku = key_of(u), nu = L.nc[u];
        const T xu = L.x[u], yu = L.y[u];
        T vxu = L.vx[u], vyu = L.vy[u];
        for (int a = 0; a < nu; ++a) {
          const int t = L.ct[a][u];
          if (L.pid[t] < pu) continue;
          T dx, dy;
          Pos<P>::sep(k, ku, xu, yu, key_of(t), L.x[t], L.y[t], dx, dy);
          T vxw = L.vx[t], vyw = L.vy[t];
          if (pair_core<P>(k, dx, dy, vxu, vyu, vxw, vyw)) {
            L.vx[t] = vxw;
            L.vy[t] = vyw;
            ++ncoll;
          }
        }
        nwall += Pos<P>::walls_key(k, ku, xu, yu, vxu, vyu);
        L.vx[u] = vxu;
        L.vy[u] = vyu;
      }
      for (int i = 0; i < m; ++i) {  // every member's final velocity
        const int u = L.sorted[base + i], s = slot_of(u);
        pt.vx[s] = L.vx[u];
        pt.vy[s] = L.vy[u];
      }
    }
    __syncthreads();
    // 5. the tile's particles: marks, wall passes of the contact-free, and the
    // row path's inputs for the rest
    for (int q = tid; q < M; q += BLOCK) {
      const int lc = L.cell[q];
      if (!in_tile(lc)) continue;
      const int s = slot_of(q), pq = L.pid[q];
      if (L.res[q]) {
        done[s] = DONE_WHOLE;
        for (int a = 0; a < L.nc[q]; ++a) npair += L.pid[L.ct[a][q]] > pq;
        continue;
      }
      if (L.ntot[q] == 0) {  // no contact: the wall pass alone
        T vx = L.vx[q], vy = L.vy[q];
        const int hw = Pos<P>::walls_key(k, key_of(q), L.x[q], L.y[q], vx, vy);
        if (hw) {
          pt.vx[s] = vx;
          pt.vy[s] = vy;
          nwall += hw;
        }
        done[s] = DONE_WHOLE;
        continue;
      }
      // the neighbour row: every contact, sorted by index, as k_contacts writes it
      ++nleft;
      const AdjRow row = adj.row(s);
      const T x = L.x[q], y = L.y[q];
      int cnt = 0, lowest = 0x7fffffff;
      bool over = false;
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
          const int nb = lc + oy * S::LW + ox;
          const int t1 = L.lstart[nb + 1];
          for (int t = L.lstart[nb]; t < t1; ++t) {
            if (t == q) continue;
            T dx, dy;
            Pos<P>::sep_nb(k, ox, oy, x, y, L.x[t], L.y[t], dx, dy);
            if (!(dx * dx + dy * dy <= dd)) continue;
            const int pt_ = L.pid[t];
            npair += pt_ > pq;
            lowest = min(lowest, pt_);
            if (cnt == KMAX) {
              over = true;
              continue;
            }
            const long long e = ((long long)pt_ << 32) | (unsigned)slot_of(t);
            int j = cnt;
            while (j > 0 && row[j - 1] > e) {
              row[j] = row[j - 1];
              --j;
            }
            row[j] = e;
            ++cnt;
          }
        }
      if (over) atomicOr(&k.flags[FLAG_CAPACITY], 1);
      deg[s] = cnt;
      done[s] = 0;
      chunk_busy[pq / RES_CHUNK] = 1;
      if (lowest > pq) {  // a candidate root for the cluster kernel
        roots[atomicAdd(&need_sweep[1], 1)] = ((long long)pq << 32) | (unsigned)s;
      }
    }
  } else {
    // the tile holds more particles than LDS: every particle of it takes the
    // row path, through the contact kernel's rows
    for (int r = 0; r < h; ++r) {
      const int g0 = (y0 + r) * k.nx + x0;
      const int a = cs[g0], b = cs[g0 + w];
      for (int s = a + tid; s < b; s += BLOCK) {
        st_row_global<P>(pt, cs, k, adj, deg, done, chunk_busy, roots, &need_sweep[1], s, npair, nwall);
        ++nleft;
      }
    }
  }
  const long long tp = block_sum_ll(npair, sh);
  const long long tc = block_sum_ll(ncoll, sh);
  const long long tw = block_sum_ll(nwall, sh);
  const long long tl = block_sum_ll(nleft, sh);
  if (tid == 0) {
    tpart[bidx] = tp;
    tpart[ntiles + bidx] = tc;
    tpart[2 * ntiles + bidx] = tw;
    tpart[3 * ntiles + bidx] = tl;
  }
}

template <int P, int TW, int TH>
__global__ __launch_bounds__(BLOCK) void k_spheres_tile(Parts<typename Prec<P>::T> pt, const int32_t *__restrict__ cs,
                                                        Consts<typename Prec<P>::T> k, Adj adj,
                                                        int32_t *__restrict__ deg, int32_t *__restrict__ done,
                                                        int32_t *ticket, int32_t *need_sweep,
                                                        int32_t *__restrict__ chunk_busy, long long *__restrict__ roots,
                                                        long long *__restrict__ tpart) {
  spheres_tile_body<P, TW, TH>(xcd_block<XCD_RUN_CONTACTS>(blockIdx.x, gridDim.x), pt, cs, k, adj, deg, done, ticket,
                               need_sweep, chunk_busy, roots, tpart, (int)gridDim.x);
}

}  // namespace lbdps
