// Batching: many independent beds advance together, one launch per phase of
// the step for all of them.  Every bed keeps its own lattice, boundary faces,
// inlet profile, parameters, particles and workspace; a table in device memory
// holds each bed's constants and buffer addresses.  The workgroups of a phase
// are the concatenation of every bed's workgroups for that phase: bed b owns
// workgroups off[b] .. off[b+1]-1, finds itself by binary search over off, and
// runs the single-bed code with its local workgroup index and count.
#pragma once

#include "kernels.hpp"

namespace lbdps {

enum { PH_COLLIDE = 0, PH_DRAG, PH_SCAN, PH_SCATTER, PH_CONTACTS, PH_CLUSTERS, PH_RESOLVE, PH_COUNT };

template <int P> struct BedArgs {
  using T = typename Prec<P>::T;
  using S = typename Prec<P>::S;
  Consts<T> k;
  S *f[2];
  int32_t *key[2], *pid[2];
  T *px[2], *py[2], *vx[2], *vy[2];
  Fields<T> fl;
  const T *lut, *inlet;
  int32_t *cs, *count, *stay, *rank, *slot, *flags, *deg, *done, *ticket, *chunk_busy, *need_sweep, *rcount;
  long long *roots;
  Adj adj;
  long long *pair_part, *wall0_part, *coll_part, *wall_part, *collc_part, *wallc_part;
  TileSums ts;
  int cf;        // population buffer holding the state when the table was written
  int cp;        // particle record set holding the state when the table was written
  int cp_moves;  // 1 if the bed has particles (its records change sets every step)
  int nlists;    // candidate-root lists of the contact kernel (its workgroups)
  __device__ Parts<T> parts(int b) const { return Parts<T>{key[b], pid[b], px[b], py[b], vx[b], vy[b]}; }
};

// Largest b in [0, nbeds) with off[b] <= blk (off[0] = 0; empty beds have
// off[b] = off[b+1] and are skipped).
__device__ __forceinline__ int bed_of(const int *__restrict__ off, int nbeds, int blk) {
  int lo = 0, hi = nbeds;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= blk) lo = mid;
    else hi = mid;
  }
  return lo;
}

// flip = parity of the step within the batched sequence: the population
// buffers swap every step, the particle record sets every step of a bed with
// particles.
#define LBDPS_BED_PROLOGUE(RUN)                                   \
  const int gb = xcd_block<RUN>(blockIdx.x, gridDim.x);          \
  const int b = bed_of(off, nbeds, gb);                           \
  const BedArgs<P> &a = tab[b];                                   \
  const int bid = gb - off[b], nbk = off[b + 1] - off[b];         \
  const int cf = a.cf ^ flip, cp = a.cp ^ (flip & a.cp_moves);    \
  (void)cf;                                                       \
  (void)cp;

template <int P>
__global__ __launch_bounds__(BLOCK) void kb_collide(const BedArgs<P> *__restrict__ tab, const int *__restrict__ off,
                                                    int nbeds, int flip) {
  LBDPS_BED_PROLOGUE(XCD_RUN_COLLIDE)
  collide_body<P>(bid, nbk, a.f[cf], a.f[1 - cf], a.fl, a.cs, a.parts(cp), a.lut, a.inlet, a.k, nullptr, nullptr,
                  nullptr);
}

template <int P, int TX>
__global__ __launch_bounds__(BLOCK) LBDPS_WAVES8 void kb_drag(const BedArgs<P> *__restrict__ tab,
                                                              const int *__restrict__ off, int nbeds, int flip) {
  LBDPS_BED_PROLOGUE(XCD_RUN_DRAG)
  drag_body_cells<P, TX>(bid, nbk, a.parts(cp), a.fl, a.cs, a.lut, a.k, a.count, a.rank, a.flags, nullptr, nullptr,
                         nullptr, a.ts, a.stay);
}
template <int P, int TX>
__global__ __launch_bounds__(BLOCK) LBDPS_WAVES6 void kb_drag_flat(const BedArgs<P> *__restrict__ tab, const int *__restrict__ off,
                                                      int nbeds, int flip) {
  LBDPS_BED_PROLOGUE(XCD_RUN_DRAG)
  drag_body_flat<P, TX>(bid, nbk, a.parts(cp), a.fl, a.cs, a.lut, a.k, a.count, a.rank, a.flags, nullptr, nullptr,
                        nullptr, a.ts, a.stay);
}

template <int P>
__global__ __launch_bounds__(BLOCK) void kb_scan(const BedArgs<P> *__restrict__ tab, const int *__restrict__ off,
                                                 int nbeds, int flip) {
  LBDPS_BED_PROLOGUE(XCD_RUN_SCAN)
  scan_cells_body(bid, nbk, a.count, (long long)a.k.C, a.ts, a.cs, a.stay);
}

template <int P>
__global__ __launch_bounds__(BLOCK) void kb_scatter(const BedArgs<P> *__restrict__ tab, const int *__restrict__ off,
                                                    int nbeds, int flip) {
  LBDPS_BED_PROLOGUE(XCD_RUN_SCATTER)
  scatter_body<typename Prec<P>::T>(bid, nbk, a.parts(cp), a.parts(1 - cp), a.rank, a.cs, a.k.npart, a.slot, a.ts,
                                    a.stay);
}

// After the scatter the records are in the other set.
template <int P>
__global__ __launch_bounds__(BLOCK) LBDPS_WAVES8 void kb_contacts(const BedArgs<P> *__restrict__ tab, const int *__restrict__ off,
                                                     int nbeds, int flip) {
  LBDPS_BED_PROLOGUE(XCD_RUN_CONTACTS)
  contacts_body<P>(bid, nbk, a.parts(1 - cp), a.cs, a.k, a.adj, a.deg, a.done, a.ticket, a.flags, a.pair_part,
                   a.wall0_part, a.chunk_busy, a.need_sweep, a.roots, a.rcount);
}

template <int P>
__global__ __launch_bounds__(BLOCK) void kb_clusters(const BedArgs<P> *__restrict__ tab, const int *__restrict__ off,
                                                     int nbeds, int flip) {
  LBDPS_BED_PROLOGUE(XCD_RUN_CLUSTERS)
  resolve_clusters_body<P>(bid, nbk, a.parts(1 - cp), a.adj, a.deg, a.done, a.k, a.need_sweep, a.collc_part,
                           a.wallc_part, a.roots, a.rcount, a.nlists);
}

template <int P>
__global__ __launch_bounds__(BLOCK) void kb_resolve(const BedArgs<P> *__restrict__ tab, const int *__restrict__ off,
                                                    int nbeds, int flip) {
  LBDPS_BED_PROLOGUE(XCD_RUN_RESOLVE)
  resolve_body<P>(bid, nbk, a.parts(1 - cp), a.slot, a.adj, a.deg, a.done, a.ticket, a.k, a.flags, a.coll_part,
                  a.wall_part, a.chunk_busy, a.need_sweep);
}

#undef LBDPS_BED_PROLOGUE

}  // namespace lbdps
