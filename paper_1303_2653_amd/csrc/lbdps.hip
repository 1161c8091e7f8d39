// Host runtime and C ABI of the lbdps library (see include/lbdps.h).
// Builds the per-count drag/porosity table in FP64, carves the caller's
// workspace, and enqueues the kernels of kernels.hpp on the context's stream.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <new>
#include <string>
#include <vector>

#include <hip/hip_ext.h>

#include "batch.hpp"
#include "coupled3d.hpp"
#include "kernels.hpp"
#include "lattice3d.hpp"
#include "lbdps.h"
#include "spheres_tile.hpp"

using namespace lbdps;

namespace {

thread_local std::string g_err;

lbdps_status fail(lbdps_status s, const std::string &m) {
  g_err = m;
  return s;
}

constexpr double kPi = 3.14159265358979323846;
constexpr int NB_CONS = 512;  // workgroups of the conservation reductions

// Scratch of lbdps_conservation_noalloc: the conservation reduction's
// per-workgroup partial sums (NB_CONS x 3 for the populations, NB_CONS x 2
// for the particles), its six outputs and its non-finite flag, in a
// library-static device array instead of a context's workspace.  The
// reduction runs on a fixed grid of NB_CONS workgroups whatever the bed, so
// this size serves every context.  Each GPU the library runs on holds its own
// copy until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns on that device (the array's name in host code is
// a host-side stand-in, not a device address).
constexpr size_t NOALLOC_PC = 0, NOALLOC_PP = NOALLOC_PC + (size_t)NB_CONS * 3,
                 NOALLOC_OUT = NOALLOC_PP + (size_t)NB_CONS * 2, NOALLOC_FLAG = NOALLOC_OUT + 8;
constexpr size_t NOALLOC_SCRATCH_BYTES = NOALLOC_FLAG * sizeof(double) + 256;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[NOALLOC_MAX_DEVICES] = {};

// Device address of `scratch` on device `dev`, looked up once per device with
// that device current (the caller's current device is restored).
lbdps_status scratch_address(int dev, void **out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(LBDPS_E_DEVICE, "device index beyond the scratch table");
  if (!g_scratch_dev[dev]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(LBDPS_E_DEVICE, "hipGetDevice failed");
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return fail(LBDPS_E_DEVICE, "hipSetDevice failed");
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr)
      return fail(LBDPS_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return LBDPS_OK;
}

int nblocks(long long n) { return (int)((n + BLOCK - 1) / BLOCK); }
// The drag kernel's flat form pays once the grid needs more than one round of
// resident workgroups (about 8 per CU on 256 CUs).
constexpr int DRAG_FLAT_MIN = 2048;
bool drag_flat(long long tiles) { return tiles > DRAG_FLAT_MIN; }
// Workgroups of the cluster resolution for n particles: each takes at least
// `lists` of the contact kernel's candidate lists and at most BLOCK; at most
// `groups_max` workgroups unless more are needed for that.
int cluster_blocks(long long n, int lists = RC_LISTS, int groups_max = RC_GROUPS_MAX) {
  const long long nl = std::max(1ll, (long long)nblocks(n));
  const long long want = std::min((nl + lists - 1) / lists, (long long)groups_max);
  return (int)std::max(std::max(want, 1ll), (nl + BLOCK - 1) / BLOCK);
}

size_t pop_bytes(int prec) { return prec == PREC_FP64 ? 8 : (prec == PREC_FP32 ? 4 : 2); }
size_t real_bytes(int prec) { return prec == PREC_FP64 ? 8 : 4; }

// Number of rows of the per-count table: every count from the first one whose
// 2-D solid fraction reaches the packing limit on shares that row.
int lut_rows(double d) {
  const double disc = kPi * d * d / 4.0;
  const double cap = kPi / (2.0 * std::sqrt(3.0));
  return (int)std::floor(cap / disc) + 2;
}

// Eq. 20 (EMMS correction), breakpoints in the lower branch.
double omega_emms(double eg) {
  if (eg <= 0.82) {
    const double t = eg - 0.7463;
    return 0.0214 / (4.0 * t * t + 0.0044) - 0.5760;
  }
  if (eg <= 0.97) {
    const double t = eg - 0.7789;
    return 0.0038 / (4.0 * t * t + 0.0040) - 0.0101;
  }
  return 32.8295 * eg - 31.8295;
}

double gas_mu(const lbdps_params &p) { return p.rho_g * ((p.tau - 0.5) / 3.0); }

// Per-count table in FP64 (columns L_* of device.hpp): porosities (Eqs. 10, 11,
// clamped at the densest disc packing), gamma (Eq. 9), omega (Eq. 20) and the
// count-dependent factors of the drag laws (Eqs. 19, 21, 22).
std::vector<double> build_lut(const lbdps_params &p) {
  const int rows = lut_rows(p.d_p);
  std::vector<double> L((size_t)rows * LUT_W, 0.0);
  const double d = p.d_p;
  const double disc = kPi * d * d / 4.0;
  const double cap = kPi / (2.0 * std::sqrt(3.0));
  const double coeff = std::sqrt(2.0) / std::sqrt(kPi * std::sqrt(3.0));
  const double mu = gas_mu(p);
  for (int n = 0; n < rows; ++n) {
    double es2 = (double)n * disc;
    if (es2 > cap) es2 = cap;
    const double e2 = 1.0 - es2;
    const double es3 = coeff * std::pow(es2, 1.5);
    const double eg = 1.0 - es3;
    double om;
    if (p.omega_mode == 1)
      om = 1.0;
    else if (eg > 0.74)
      om = omega_emms(eg);
    else
      om = p.omega_dense;
    const double gam = es2 * (p.tau - 0.5) / ((1.0 - es2) + (p.tau - 0.5));
    double *r = &L[(size_t)n * LUT_W];
    r[L_ES3] = es3;
    r[L_UDIV] = p.u_gas_porosity == 0 ? e2 : (p.u_gas_porosity == 1 ? eg : 1.0);
    r[L_OMG] = om * gam;
    r[L_RELAX] = (1.0 - gam) / p.tau;
    r[L_A] = 18.0 * (1.0 - eg) * om * mu / (d * d);
    r[L_BRE] = eg * p.rho_g;
    r[L_H] = 0.75 * (1.0 - eg) * eg * p.rho_g;
    r[L_OM] = om;
    r[L_D1] = 150.0 * (1.0 - eg) * (1.0 - eg) * mu / (eg * d * d);
    r[L_D2] = 1.75 * (1.0 - eg) * p.rho_g;
    r[L_DILUTE] = eg > 0.74 ? 1.0 : 0.0;
    r[L_ES2] = es2;
  }
  return L;
}

// Particle sub-steps per lattice step (0 is taken as 1).
int n_sub_of(const lbdps_params &p) { return p.n_sub > 1 ? p.n_sub : 1; }

struct DConsts {  // FP64 master copy of the kernel constants
  double tau, d, mu, vp, m, msum, one_e, e_pw, r, geff[2], fp, halfG[2], src[Q];
  double cs18;  // 18 C_s^2 (Eq. 15)
  double h;     // particle sub-step length 1 / n_sub
};

DConsts make_dconsts(const lbdps_params &p) {
  DConsts c{};
  c.tau = p.tau;
  c.d = p.d_p;
  c.mu = gas_mu(p);
  c.vp = kPi * p.d_p * p.d_p * p.d_p / 6.0;
  c.m = p.rho_s * c.vp;
  c.msum = c.m + c.m;
  c.one_e = 1.0 + p.e_pp;
  c.e_pw = p.e_pw;
  c.r = 0.5 * p.d_p;
  c.geff[0] = (1.0 - p.rho_g / p.rho_s) * p.g[0];
  c.geff[1] = (1.0 - p.rho_g / p.rho_s) * p.g[1];
  c.fp = (double)p.pressure_force_sign * c.vp;
  c.cs18 = 18.0 * p.cs_smag * p.cs_smag;
  c.h = 1.0 / (double)n_sub_of(p);
  c.halfG[0] = 0.5 * p.body_force[0];
  c.halfG[1] = 0.5 * p.body_force[1];
  for (int i = 0; i < Q; ++i)
    c.src[i] = 3.0 * wgt<double>(i) * (cx_of(i) * p.body_force[0] + cy_of(i) * p.body_force[1]);
  return c;
}

// Cell-start scan tile: SCAN_TILE = 2^shift cells.
int cell_tile_shift(size_t) {
  int shift = 0;
  while ((1 << shift) < SCAN_TILE) ++shift;
  return shift;
}

// Workspace layout: every buffer 256-byte aligned.
struct Carver {
  char *base;
  size_t off = 0;
  template <class X> X *take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    X *p = base ? reinterpret_cast<X *>(base + off) : nullptr;
    off += (count > 0 ? count : 1) * sizeof(X);
    return p;
  }
};

}  // namespace

struct lbdps_ctx {
  lbdps_params p{};
  int prec = 0, nx = 0, ny = 0, C = 0, nlut = 0;
  long long nmax = 0, n = 0;
  hipStream_t stream = nullptr;
  unsigned long long *cross = nullptr;  // device: running net count of outlet crossings
  unsigned long long *hist = nullptr;   // device: particles-per-cell histogram
  unsigned long long cross_seen = 0;    // its value at the previous lbdps_outlet_crossings
  long long cross_step0 = 0;            // the step counter then
  int device = 0;           // the HIP device current at creation
  void *scratch = nullptr;  // that device's address of the static scratch array
  int cf = 0, cp = 0;
  bool bins_valid = false;
  long long step = 0;
  bool in_batch = false;  // owned by a batch: destroyed with it
  lbdps_tuning tune{RC_LISTS, RC_GROUPS_MAX, 0, 0};
  int sphere_tiles = 0;  // tiles of the tile kernel in the most recent collision stage (0: not used)
  int drag_blocks = 0;  // drag workgroups of the most recent step (its partial sums)
  int cluster_groups() const { return cluster_blocks(n, tune.cluster_lists, tune.cluster_groups_max); }
  DConsts dc{};
  // device buffers (carved from the workspace)
  void *f[2]{};
  void *fld[7]{};  // rho, ugx, ugy, beta, fpgx, fpgy, es
  int32_t *count = nullptr, *stay = nullptr, *cs = nullptr, *spart = nullptr;
  int32_t *key[2]{}, *pid[2]{};
  void *px[2]{}, *py[2]{}, *vx[2]{}, *vy[2]{};
  int32_t *rank = nullptr, *perm = nullptr, *slot = nullptr, *deg = nullptr, *done = nullptr;
  int32_t *ticket = nullptr, *flags = nullptr, *nonfinite = nullptr;
  long long *adj_in = nullptr, *adj_ov = nullptr;
  Adj adj() const { return Adj{adj_in, adj_ov}; }
  void *lut = nullptr, *inlet = nullptr;
  long long *pair_part = nullptr, *coll_part = nullptr, *wall_part = nullptr, *wall0_part = nullptr,
            *zero_part = nullptr;
  int32_t *tile_sum = nullptr, *chunk_busy = nullptr, *need_sweep = nullptr;
  int tile_shift = 11;
  long long *roots = nullptr;
  int32_t *rcount = nullptr;
  long long *collc_part = nullptr, *wallc_part = nullptr;
  long long *tile_part = nullptr;  // the tile kernel's pairs, collisions, wall hits and particles left, per tile
  int ntiles = 0;
  double *cons_pc = nullptr, *cons_pp = nullptr, *cons_out = nullptr;
  double *diag_pc = nullptr, *diag_pp = nullptr, *diag_out = nullptr;  // the periodic check's own sums
  int32_t *diag_flag = nullptr;
  long long diag_step = -1;  // step after which the latest periodic check ran
  double *eg_tab = nullptr;        // FP64 gas voidage per particle count (Eq. 11), for lbdps_voidage
  long long *obs_part = nullptr;   // per-workgroup partial counts of lbdps_voidage
  int32_t *dg_n = nullptr;
  void *dg_vsx = nullptr, *dg_vsy = nullptr, *dg_fdx = nullptr, *dg_fdy = nullptr;
  void *acx = nullptr, *acy = nullptr;  // accelerations held over the lattice step (n_sub > 1)
  // per-kernel event timing
  uint32_t timed = 0;
  struct Mark {
    hipEvent_t a, b;
    int k;
    bool extra;  // a further launch of the same phase: its time adds, its launch does not count
  };
  std::vector<Mark> marks;
  size_t nmarks = 0;
  double ms[LBDPS_K_COUNT] = {0};
  long long launches[LBDPS_K_COUNT] = {0};
  ~lbdps_ctx() {
    for (auto &m : marks) {
      (void)hipEventDestroy(m.a);
      (void)hipEventDestroy(m.b);
    }
  }
};

namespace {

size_t carve(const lbdps_params &p, long long nmax, char *base, lbdps_ctx *x) {
  Carver cv{base};
  const size_t C = (size_t)p.nx * p.ny;
  const size_t N = (size_t)nmax;
  const size_t sS = pop_bytes(p.precision), sT = real_bytes(p.precision);
  const size_t tiles = (std::max(C + 1, N + 1) + SCAN_TILE - 1) / SCAN_TILE + 1;
  auto raw = [&](size_t bytes) { return cv.take<char>(bytes); };
  char *f0 = raw(Q * C * sS), *f1 = raw(Q * C * sS);
  char *fl[7];
  for (auto &q : fl) q = raw(C * sT);
  int32_t *count = cv.take<int32_t>(C), *stay = cv.take<int32_t>(C), *cs = cv.take<int32_t>(C + 1);
  int32_t *spart = cv.take<int32_t>(tiles);
  int32_t *key[2], *pid[2];
  char *px[2], *py[2], *vx[2], *vy[2];
  for (int b = 0; b < 2; ++b) {
    key[b] = cv.take<int32_t>(N);
    pid[b] = cv.take<int32_t>(N);
    px[b] = raw(N * sT);
    py[b] = raw(N * sT);
    vx[b] = raw(N * sT);
    vy[b] = raw(N * sT);
  }
  int32_t *rank = cv.take<int32_t>(N + 1), *perm = cv.take<int32_t>(N + 1), *slot = cv.take<int32_t>(N);
  int32_t *deg = cv.take<int32_t>(N), *done = cv.take<int32_t>(N);
  long long *adj_in = cv.take<long long>(N * ADJ_IN), *adj_ov = cv.take<long long>(N * (KMAX - ADJ_IN));
  int32_t *ticket = cv.take<int32_t>(4), *flags = cv.take<int32_t>(FLAG_COUNT), *nonfinite = cv.take<int32_t>(4);
  char *lut = raw((size_t)lut_rows(p.d_p) * LUT_W * sT), *inlet = raw((size_t)p.nx * sT);
  const size_t nbN = (size_t)nblocks((long long)N), nbC = (size_t)nblocks((long long)C);
  size_t ndrag = 0;  // drag workgroups of the tile shape with the most of them
  for (int t = 0; t < DRAG_TILES; ++t) {
    const int w = drag_tile_w(t), h = BLOCK / w;
    ndrag = std::max(ndrag, (size_t)((p.nx + w - 1) / w) * ((p.ny + h - 1) / h));
  }
  const size_t ntile2 = ndrag;
  long long *pair_part = cv.take<long long>(std::max(nbN, ntile2)), *coll_part = cv.take<long long>(nbN);
  long long *wall_part = cv.take<long long>(nbN), *zero_part = cv.take<long long>(std::max(nbC, ndrag));
  long long *wall0_part = cv.take<long long>(std::max(nbN, ntile2));
  const int shift = cell_tile_shift(C);
  const size_t ntiles = (C + ((size_t)1 << shift) - 1) >> shift;
  int32_t *tile_sum = cv.take<int32_t>(ntiles + 1);
  long long *roots = cv.take<long long>(nbN * BLOCK);
  int32_t *rcount = cv.take<int32_t>(nbN);
  int32_t *chunk_busy = cv.take<int32_t>(N / RES_CHUNK + 1), *need_sweep = cv.take<int32_t>(4);
  long long *collc_part = cv.take<long long>(nbN), *wallc_part = cv.take<long long>(nbN);
  size_t nst = 1;  // tiles of the sphere tile shape with the most of them
  for (int t = 1; t < SPHERE_TILES; ++t) {
    int tw, th;
    sphere_tile_dims(t, tw, th);
    nst = std::max(nst, (size_t)st_tiles(p.nx, p.ny, tw, th));
  }
  long long *tile_part = cv.take<long long>(4 * nst);
  double *pc = cv.take<double>(NB_CONS * 3), *pp = cv.take<double>(NB_CONS * 2), *co = cv.take<double>(8);
  double *dpc = cv.take<double>(NB_CONS * 3), *dpp = cv.take<double>(NB_CONS * 2), *dco = cv.take<double>(8);
  int32_t *dfl = cv.take<int32_t>(4);
  double *egt = cv.take<double>((size_t)lut_rows(p.d_p));
  long long *obs = cv.take<long long>((size_t)nblocks(p.nx) + 1);
  unsigned long long *cross = cv.take<unsigned long long>(1);
  unsigned long long *hist = cv.take<unsigned long long>(HIST_BINS_MAX);
  int32_t *dg_n = nullptr;
  char *dvx = nullptr, *dvy = nullptr, *dfx = nullptr, *dfy = nullptr;
  if (p.diagnostics) {
    dg_n = cv.take<int32_t>(C);
    dvx = raw(C * sT);
    dvy = raw(C * sT);
    dfx = raw(N * sT);
    dfy = raw(N * sT);
  }
  char *acx = nullptr, *acy = nullptr;
  if (n_sub_of(p) > 1 || p.diagnostics) {
    acx = raw(N * sT);
    acy = raw(N * sT);
  }
  if (x) {
    x->f[0] = f0;
    x->f[1] = f1;
    for (int i = 0; i < 7; ++i) x->fld[i] = fl[i];
    x->count = count;
    x->stay = stay;
    x->cs = cs;
    x->spart = spart;
    for (int b = 0; b < 2; ++b) {
      x->key[b] = key[b];
      x->pid[b] = pid[b];
      x->px[b] = px[b];
      x->py[b] = py[b];
      x->vx[b] = vx[b];
      x->vy[b] = vy[b];
    }
    x->rank = rank;
    x->perm = perm;
    x->slot = slot;
    x->deg = deg;
    x->done = done;
    x->adj_in = adj_in;
    x->adj_ov = adj_ov;
    x->ticket = ticket;
    x->flags = flags;
    x->nonfinite = nonfinite;
    x->lut = lut;
    x->inlet = inlet;
    x->pair_part = pair_part;
    x->coll_part = coll_part;
    x->wall_part = wall_part;
    x->zero_part = zero_part;
    x->wall0_part = wall0_part;
    x->tile_sum = tile_sum;
    x->tile_shift = shift;
    x->roots = roots;
    x->rcount = rcount;
    x->chunk_busy = chunk_busy;
    x->need_sweep = need_sweep;
    x->collc_part = collc_part;
    x->tile_part = tile_part;
    x->wallc_part = wallc_part;
    x->ntiles = (int)ntiles;
    x->cons_pc = pc;
    x->cons_pp = pp;
    x->cons_out = co;
    x->diag_pc = dpc;
    x->diag_pp = dpp;
    x->diag_out = dco;
    x->diag_flag = dfl;
    x->eg_tab = egt;
    x->obs_part = obs;
    x->cross = cross;
    x->hist = hist;
    x->dg_n = dg_n;
    x->dg_vsx = dvx;
    x->dg_vsy = dvy;
    x->dg_fdx = dfx;
    x->dg_fdy = dfy;
    x->acx = acx;
    x->acy = acy;
  }
  return cv.off + 256;
}

// Start / stop the event bracket of kernel k if it is being timed.
void tstart(lbdps_ctx *x, int k) {
  if (!(x->timed >> k & 1u)) return;
  if (x->nmarks == x->marks.size()) {
    lbdps_ctx::Mark m{};
    if (hipEventCreate(&m.a) != hipSuccess || hipEventCreate(&m.b) != hipSuccess) return;
    x->marks.push_back(m);
  }
  x->marks[x->nmarks].k = k;
  x->marks[x->nmarks].extra = false;
  (void)hipEventRecord(x->marks[x->nmarks].a, x->stream);
}
void tstop(lbdps_ctx *x, int k) {
  if (!(x->timed >> k & 1u) || x->nmarks >= x->marks.size() || x->marks[x->nmarks].k != k) return;
  (void)hipEventRecord(x->marks[x->nmarks].b, x->stream);
  x->nmarks += 1;
}

// Launches a step kernel on x's stream.  When its phase k is being timed, the
// launch carries a pair of events that the dispatch itself stamps at the
// kernel's start and end, so the time is the kernel's own (an event pair
// recorded around a launch also counts the queue's work between them, a few
// microseconds).  extra: a further launch of the same phase.
template <typename F, typename... Args>
void tlaunch(lbdps_ctx *x, int k, bool extra, F kern, dim3 grid, Args... args) {
  hipEvent_t a = nullptr, b = nullptr;
  if (x->timed >> k & 1u) {
    if (x->nmarks == x->marks.size()) {
      lbdps_ctx::Mark m{};
      if (hipEventCreate(&m.a) == hipSuccess && hipEventCreate(&m.b) == hipSuccess) x->marks.push_back(m);
    }
    if (x->nmarks < x->marks.size()) {
      lbdps_ctx::Mark &m = x->marks[x->nmarks++];
      m.k = k;
      m.extra = extra;
      a = m.a;
      b = m.b;
    }
  }
  if (a)
    hipExtLaunchKernelGGL(kern, grid, dim3(BLOCK), 0, x->stream, a, b, 0, args...);
  else
    hipLaunchKernelGGL(kern, grid, dim3(BLOCK), 0, x->stream, args...);
}

lbdps_status check_hip(hipError_t e, const char *what) {
  if (e == hipSuccess) return LBDPS_OK;
  return fail(LBDPS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

lbdps_status launch_status(const char *what) { return check_hip(hipGetLastError(), what); }

template <int P> struct Impl {
  using T = typename Prec<P>::T;
  using S = typename Prec<P>::S;

  static Consts<T> consts(const lbdps_ctx *x) {
    Consts<T> k{};
    const DConsts &d = x->dc;
    k.nx = x->nx;
    k.ny = x->ny;
    k.C = x->C;
    k.nlut = x->nlut;
    {  // key / nx by multiplication (see cell_row)
      int l = 0;
      while ((1ll << l) < x->nx) ++l;
      k.nx_s = 31 + l;
      k.nx_m = (unsigned long long)(((1ull << k.nx_s) + (unsigned long long)x->nx - 1) / (unsigned long long)x->nx);
    }
    k.per_x = x->p.bc[0] == BC_PERIODIC;
    k.gas_per_y = x->p.bc[2] == BC_PERIODIC;
    k.per_y = k.gas_per_y || x->p.particles_periodic_y != 0;  // the circulating loop
    k.bc_ylo = x->p.bc[2];
    k.bc_yhi = x->p.bc[3];
    k.drag_abs = x->p.drag_ratio_mode == 1;
    k.drag_reg = x->p.drag_ratio_mode == 2;
    k.npart = (int)x->n;
    k.tau = (T)d.tau;
    k.d = (T)d.d;
    k.mu = (T)d.mu;
    k.vp = (T)d.vp;
    k.m = (T)d.m;
    k.msum = (T)d.msum;
    k.one_e = (T)d.one_e;
    k.e_pw = (T)d.e_pw;
    k.r = (T)d.r;
    k.les = x->p.cs_smag != 0.0;
    k.cs18 = (T)d.cs18;
    for (int a = 0; a < 2; ++a) {
      k.geff[a] = (T)d.geff[a];
      k.halfG[a] = (T)d.halfG[a];
    }
    k.fp = (T)d.fp;
    for (int i = 0; i < Q; ++i) k.src[i] = (T)d.src[i];
    k.h = (T)d.h;
    k.acx = (T *)x->acx;
    k.acy = (T *)x->acy;
    k.spin_limit = 1u << 22;
    k.flags = x->flags;
    k.cross = x->cross;
    return k;
  }
  static Parts<T> parts(const lbdps_ctx *x, int b) {
    return Parts<T>{x->key[b], x->pid[b], (T *)x->px[b], (T *)x->py[b], (T *)x->vx[b], (T *)x->vy[b]};
  }
  static Fields<T> fields(const lbdps_ctx *x) {
    return Fields<T>{(T *)x->fld[0], (T *)x->fld[1], (T *)x->fld[2], (T *)x->fld[3],
                     (T *)x->fld[4], (T *)x->fld[5], (T *)x->fld[6]};
  }

  static void scan(lbdps_ctx *x, int32_t *in, long long n, int32_t *out, int zero_in) {
    const int tiles = (int)((n + SCAN_TILE - 1) / SCAN_TILE) + (n == 0);
    hipLaunchKernelGGL(k_scan_reduce, dim3(tiles), dim3(BLOCK), 0, x->stream, in, n, x->spart);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(BLOCK), 0, x->stream, x->spart, tiles, out + n);
    hipLaunchKernelGGL(k_scan_apply, dim3(tiles), dim3(BLOCK), 0, x->stream, in, n, x->spart, out, zero_in);
  }

  static TileSums tiles(const lbdps_ctx *x) { return TileSums{x->tile_sum, x->ntiles, x->tile_shift}; }
  // Drag workgroups for tile shape t (the context's own by default).
  static int drag_tiles(const lbdps_ctx *x, int t = -1) {
    const int w = drag_tile_w(t < 0 ? x->tune.drag_tile : t), h = BLOCK / w;
    return ((x->nx + w - 1) / w) * ((x->ny + h - 1) / h);
  }
  // The drag kernel of tile shape t, flat or one thread per cell.
  using DragKern = void (*)(Parts<T>, Fields<T>, const int32_t *, const T *, Consts<T>, int32_t *, int32_t *,
                            int32_t *, T *, T *, long long *, TileSums, int32_t *);
  static DragKern drag_kernel(int t, bool flat) {
    switch (t) {
      case 1: return flat ? k_drag_flat<P, 64> : k_drag<P, 64>;
      case 2: return flat ? k_drag_flat<P, 128> : k_drag<P, 128>;
      default: return flat ? k_drag_flat<P, 32> : k_drag<P, 32>;
    }
  }
  // Workgroups of the resolution: they loop over chunks of particle indices.
  static int resolve_blocks(const lbdps_ctx *x) {
    const long long chunks = (x->n + RES_CHUNK - 1) / RES_CHUNK;
    return (int)std::max(1ll, std::min(chunks, 512ll));
  }

  // Counting sort of the particle storage by cell: the per-cell counts are in
  // x->count (slots in x->rank) and the tile sums in x->tile_sum; cell starts
  // in one pass, then every record moves to its slot in the other storage.
  // Each cell's segment is put in particle-index order by the next collision.
  static void sort_counted(lbdps_ctx *x, bool tile_sums = true, bool extra = false) {
    if (tile_sums) {
      tlaunch(x, LBDPS_K_SCAN, extra, k_scan_cells, dim3(x->ntiles), x->count, (long long)x->C, tiles(x), x->cs,
              (const int32_t *)x->stay);
    } else {
      tstart(x, LBDPS_K_SCAN);
      scan(x, x->count, x->C, x->cs, 1);
      tstop(x, LBDPS_K_SCAN);
    }
    const int N = (int)x->n;
    tlaunch(x, LBDPS_K_SCATTER, extra, k_scatter<T>, dim3(std::max(nblocks(N), 1)), parts(x, x->cp),
            parts(x, 1 - x->cp), (const int32_t *)x->rank, (const int32_t *)x->cs, N, x->slot, tiles(x),
            (const int32_t *)x->stay);
    x->cp = 1 - x->cp;
  }

  static void rebin(lbdps_ctx *x) {
    const int N = (int)x->n;
    // every particle counts as an arrival: no cell has stayers
    hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(x->C)), dim3(BLOCK), 0, x->stream, x->stay, (long long)x->C, 0);
    if (N > 0)
      hipLaunchKernelGGL(k_bin, dim3(nblocks(N)), dim3(BLOCK), 0, x->stream, x->key[x->cp], N, x->count, x->rank);
    sort_counted(x, false);
    x->bins_valid = true;
  }

  // extra: a further sub-step of the same lattice step (its launches add time,
  // not launch counts)
  using TileKern = void (*)(Parts<T>, const int32_t *, Consts<T>, Adj, int32_t *, int32_t *, int32_t *, int32_t *,
                            int32_t *, long long *, long long *);
  static TileKern tile_kernel(int t) {
    switch (t) {
      case 2: return k_spheres_tile<P, 16, 16>;
      case 3: return k_spheres_tile<P, 64, 4>;
      default: return k_spheres_tile<P, 32, 8>;
    }
  }
  static int sphere_tiles(const lbdps_ctx *x, int t) {
    int tw, th;
    sphere_tile_dims(t, tw, th);
    return st_tiles(x->nx, x->ny, tw, th);
  }
  // The collision stage (A6 + A7).  With a sphere tile shape, the tile kernel
  // finds the contacts and resolves the clusters that lie within its tiles'
  // reach, and writes rows and one compact root list only for the rest,
  // which the cluster kernel and the ordered sweep then take as before.
  static void hard_spheres(lbdps_ctx *x, bool extra = false) {
    const int N = (int)x->n;
    if (N == 0) return;
    const Consts<T> k = consts(x);
    const int st = x->tune.sphere_tile;
    x->sphere_tiles = st > 0 ? sphere_tiles(x, st) : 0;
    if (st > 0) {
      tlaunch(x, LBDPS_K_CONTACTS, extra, tile_kernel(st), dim3(x->sphere_tiles), parts(x, x->cp),
              (const int32_t *)x->cs, k, x->adj(), x->deg, x->done, x->ticket, x->need_sweep, x->chunk_busy,
              x->roots, x->tile_part);
    } else {
      tlaunch(x, LBDPS_K_CONTACTS, extra, nblocks(N) <= CONTACTS_SMALL_MAX ? k_contacts_small<P> : k_contacts<P>,
              dim3(nblocks(N)), parts(x, x->cp), (const int32_t *)x->cs, k,
              x->adj(), x->deg, x->done, x->ticket, x->flags, x->pair_part, x->wall0_part, x->chunk_busy,
              x->need_sweep, x->roots, x->rcount);
    }
    tlaunch(x, LBDPS_K_RESOLVE, extra, k_resolve_clusters<P>, dim3(x->cluster_groups()), parts(x, x->cp), x->adj(),
            (const int32_t *)x->deg, x->done, k, x->need_sweep, x->collc_part, x->wallc_part,
            (const long long *)x->roots, (const int32_t *)x->rcount, nblocks(N),
            st > 0 ? (const int32_t *)x->need_sweep + 1 : nullptr);
    tlaunch(x, LBDPS_K_RESOLVE, true, k_resolve<P>, dim3(resolve_blocks(x)), parts(x, x->cp),
            (const int32_t *)x->slot, x->adj(), (const int32_t *)x->deg, x->done, x->ticket, k, x->flags,
            x->coll_part, x->wall_part, x->chunk_busy, x->need_sweep);
  }

  static lbdps_status step(lbdps_ctx *x, int nsteps) {
    const Consts<T> k = consts(x);
    const bool dg = x->p.diagnostics != 0;
    for (int it = 0; it < nsteps; ++it) {
      if (!x->bins_valid) rebin(x);
      tlaunch(x, LBDPS_K_COLLIDE, false, k_collide<P>, dim3(nblocks(x->C)), (const S *)x->f[x->cf],
              (S *)x->f[1 - x->cf], fields(x), (const int32_t *)x->cs, parts(x, x->cp), (const T *)x->lut,
              (const T *)x->inlet, k, dg ? x->dg_n : nullptr, dg ? (T *)x->dg_vsx : nullptr,
              dg ? (T *)x->dg_vsy : nullptr);
      if (x->n > 0) {
        const int nt = drag_tiles(x);
        x->drag_blocks = nt;  // the drag's per-workgroup partial sums of this step
        tlaunch(x, LBDPS_K_DRAG, false, drag_kernel(x->tune.drag_tile, drag_flat(nt)), dim3(nt), parts(x, x->cp),
                fields(x), (const int32_t *)x->cs, (const T *)x->lut, consts(x), x->count, x->rank, x->flags,
                dg ? (T *)x->dg_fdx : nullptr, dg ? (T *)x->dg_fdy : nullptr, dg ? x->zero_part : nullptr, tiles(x),
                x->stay);
        sort_counted(x);
        hard_spheres(x);
        // further particle sub-steps under the accelerations the drag kernel held
        for (int sub = 1; sub < n_sub_of(x->p); ++sub) {
          tlaunch(x, LBDPS_K_DRAG, true, k_advance<P>, dim3(nblocks(x->C)), parts(x, x->cp), consts(x),
                  (const int32_t *)x->cs, x->count, x->rank, x->stay, x->flags, tiles(x));
          sort_counted(x, true, true);
          hard_spheres(x, true);
        }
      }
      x->cf = 1 - x->cf;
      x->step += 1;
      if (x->p.diag_every > 0 && x->step % x->p.diag_every == 0) {  // the periodic FP64 check
        conservation(x, x->diag_pc, x->diag_pp, x->diag_out, x->diag_flag);
        hipLaunchKernelGGL(k_flag_nonfinite, dim3(1), dim3(64), 0, x->stream, (const double *)x->diag_out,
                           x->flags);
        x->diag_step = x->step;
      }
    }
    return launch_status("lbdps_step");
  }

  static lbdps_status voidage(lbdps_ctx *x, int y0, int y1, double thr, double *rows, double *cols,
                              int64_t *count) {
    if (!x->bins_valid) rebin(x);
    const int ncb = nblocks(x->nx);
    hipLaunchKernelGGL(k_voidage, dim3(x->ny + ncb), dim3(BLOCK), 0, x->stream, (const int32_t *)x->cs, x->nx,
                       x->ny, x->nlut, (const double *)x->eg_tab, y0, y1, thr, rows, cols, x->obs_part);
    if (count)
      hipLaunchKernelGGL(k_voidage_count, dim3(1), dim3(BLOCK), 0, x->stream, (const long long *)x->obs_part, ncb,
                         (long long *)count);
    return launch_status("lbdps_voidage");
  }

  static lbdps_status count_histogram(lbdps_ctx *x, int nbins) {
    if (!x->bins_valid) rebin(x);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(BLOCK), 0, x->stream, (int32_t *)x->hist, 2ll * nbins, 0);
    hipLaunchKernelGGL(k_count_hist, dim3(std::min(nblocks(x->C), 1024)), dim3(BLOCK), 0, x->stream,
                       (const int32_t *)x->cs, (int)x->C, nbins, x->hist);
    return launch_status("lbdps_count_histogram");
  }

  static lbdps_status collide_particles(lbdps_ctx *x) {
    if (!x->bins_valid) rebin(x);
    hard_spheres(x);
    return launch_status("lbdps_collide_particles");
  }

  // Neighbour rows and degrees of every particle at the current positions (the
  // contacts of the most recent collision stage: positions do not change
  // after it), for the pair listing; nothing else is written.
  static void rows(lbdps_ctx *x) {
    const int N = (int)x->n;
    if (!x->bins_valid) rebin(x);
    hipLaunchKernelGGL((k_contacts<P, CT_ROWS>), dim3(nblocks(N)), dim3(BLOCK), 0, x->stream, parts(x, x->cp),
                       (const int32_t *)x->cs, consts(x), x->adj(), x->deg, x->done, x->ticket, x->flags,
                       x->pair_part, x->wall0_part, x->chunk_busy, x->need_sweep, x->roots, x->rcount);
  }

  static lbdps_status set_state(lbdps_ctx *x, const double *d_f, const double *d_pos, const double *d_vel,
                                long long n) {
    const long long e = (long long)Q * x->C;
    hipLaunchKernelGGL(k_set_f<P>, dim3((unsigned)((e + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, x->stream, d_f,
                       (S *)x->f[x->cf], x->C);
    x->n = n;
    const Consts<T> k = consts(x);
    if (n > 0)
      hipLaunchKernelGGL(k_set_parts<P>, dim3(nblocks(n)), dim3(BLOCK), 0, x->stream, d_pos, d_vel, (int)n,
                         parts(x, x->cp), x->slot, k, x->flags);
    x->bins_valid = false;
    x->step = 0;
    x->diag_step = -1;  // no periodic check has run on this state
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(BLOCK), 0, x->stream, (int32_t *)x->cross, 2ll, 0);
    x->cross_seen = 0;
    x->cross_step0 = 0;
    if (x->p.diagnostics) {
      hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(x->C)), dim3(BLOCK), 0, x->stream, x->dg_n, (long long)x->C, 0);
    }
    return launch_status("lbdps_set_state");
  }

  static void get_particles(lbdps_ctx *x, double *pos, double *vel, double *fd, int32_t *cell) {
    if (x->n == 0) return;
    const Consts<T> k = consts(x);
    hipLaunchKernelGGL(k_get_parts<P>, dim3(nblocks(x->n)), dim3(BLOCK), 0, x->stream, parts(x, x->cp), x->slot,
                       (int)x->n, k, pos, vel, cell, (const T *)x->dg_fdx, (const T *)x->dg_fdy,
                       x->p.diagnostics ? fd : nullptr);
  }

  static void get_field2(lbdps_ctx *x, const void *a, const void *b, double *out, double add = 0.0) {
    hipLaunchKernelGGL(k_get_field<T>, dim3(nblocks(x->C)), dim3(BLOCK), 0, x->stream, (const T *)a, (const T *)b,
                       x->C, out, add);
  }

  static void get_f(lbdps_ctx *x, double *out) {
    const long long e = (long long)Q * x->C;
    hipLaunchKernelGGL(k_get_f<P>, dim3((unsigned)((e + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, x->stream,
                       (const S *)x->f[x->cf], out, x->C);
  }

  // The FP64 conservation sums with the given scratch: partials pc [NB_CONS][3]
  // and pp [NB_CONS][2], output out [6], flag (cleared here first).
  static void conservation(lbdps_ctx *x, double *pc, double *pp, double *out, int32_t *flag) {
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(BLOCK), 0, x->stream, flag, 1ll, 0);
    hipLaunchKernelGGL(k_cons_cells<P>, dim3(NB_CONS), dim3(BLOCK), 0, x->stream, (const S *)x->f[x->cf], x->C,
                       pc, flag);
    hipLaunchKernelGGL(k_cons_parts<T>, dim3(NB_CONS), dim3(BLOCK), 0, x->stream, (const T *)x->vx[x->cp],
                       (const T *)x->vy[x->cp], (int)x->n, x->dc.m, pp, flag);
    hipLaunchKernelGGL(k_cons_final, dim3(1), dim3(BLOCK), 0, x->stream, (const double *)pc, NB_CONS,
                       (const double *)pp, NB_CONS, (const int32_t *)flag, out);
  }
};

template <class F> lbdps_status dispatch(lbdps_ctx *x, F &&fn) {
  switch (x->prec) {
    case PREC_FP64: return fn(Impl<PREC_FP64>{});
    case PREC_FP32: return fn(Impl<PREC_FP32>{});
    case PREC_FP16DEV: return fn(Impl<PREC_FP16DEV>{});
    case PREC_BF16DEV: return fn(Impl<PREC_BF16DEV>{});
  }
  return fail(LBDPS_E_INVALID, "unknown precision");
}

// Wait for the stream and report device-side errors latched since the last sync.
lbdps_status sync_and_check(lbdps_ctx *x, const char *what) {
  lbdps_status st = check_hip(hipStreamSynchronize(x->stream), what);
  if (st != LBDPS_OK) return st;
  int32_t fl[FLAG_COUNT];
  st = check_hip(hipMemcpy(fl, x->flags, sizeof(fl), hipMemcpyDeviceToHost), what);
  if (st != LBDPS_OK) return st;
  bool any = false;
  for (int i = 0; i < FLAG_COUNT; ++i) any |= fl[i] != 0;
  if (!any) return LBDPS_OK;
  // clear the latched flags, then report the first error
  const int32_t zero[FLAG_COUNT] = {0};
  check_hip(hipMemcpy(x->flags, zero, sizeof(zero), hipMemcpyHostToDevice), what);
  const int32_t *had = fl;
  if (had[FLAG_DOMAIN])
    return fail(LBDPS_E_INVALID, std::string(what) + ": a particle left the domain or was placed outside it");
  if (had[FLAG_CAPACITY])
    return fail(LBDPS_E_CAPACITY, std::string(what) + ": a particle had more than LBDPS_MAX_CONTACTS contacts");
  if (had[FLAG_STALL]) return fail(LBDPS_E_STALL, std::string(what) + ": collision resolution exceeded its wait bound");
  if (had[FLAG_NONFINITE])
    return fail(LBDPS_E_NONFINITE, std::string(what) + ": the periodic check found a non-finite population or velocity");
  return fail(LBDPS_E_DEVICE, std::string(what) + ": unknown device flag");
}

bool is_fin(double v) { return std::isfinite(v); }

}  // namespace

extern "C" {

const char *lbdps_status_str(lbdps_status s) {
  switch (s) {
    case LBDPS_OK: return "ok";
    case LBDPS_E_INVALID: return "invalid argument";
    case LBDPS_E_SHAPE: return "shape mismatch";
    case LBDPS_E_DEVICE: return "device error";
    case LBDPS_E_UNSUPPORTED: return "unsupported";
    case LBDPS_E_NONFINITE: return "non-finite value in state";
    case LBDPS_E_CAPACITY: return "capacity exceeded";
    case LBDPS_E_STALL: return "collision resolution stalled";
  }
  return "unknown status";
}

const char *lbdps_last_error(void) { return g_err.c_str(); }

lbdps_status lbdps_validate_params(const lbdps_params *p, int64_t max_particles) {
  if (!p) return fail(LBDPS_E_INVALID, "params is NULL");
  if (p->nx < 3 || p->ny < 3) return fail(LBDPS_E_SHAPE, "nx and ny must be >= 3");
  if ((long long)p->nx * p->ny >= (1ll << 29)) return fail(LBDPS_E_SHAPE, "nx * ny must be < 2^29");
  for (int i = 0; i < 4; ++i)
    if (p->bc[i] < 0 || p->bc[i] > 3) return fail(LBDPS_E_INVALID, "bc values must be 0..3");
  if (p->bc[0] > 1 || p->bc[1] > 1) return fail(LBDPS_E_INVALID, "x faces must be PERIODIC or WALL");
  if ((p->bc[0] == 0) != (p->bc[1] == 0)) return fail(LBDPS_E_INVALID, "PERIODIC must be set on both x faces");
  if ((p->bc[2] == 0) != (p->bc[3] == 0)) return fail(LBDPS_E_INVALID, "PERIODIC must be set on both y faces");
  if (!(is_fin(p->tau) && p->tau > 0.5)) return fail(LBDPS_E_INVALID, "tau must be > 0.5");
  if (!(is_fin(p->rho_g) && p->rho_g > 0)) return fail(LBDPS_E_INVALID, "rho_g must be > 0");
  if (!(is_fin(p->rho_s) && p->rho_s > 0)) return fail(LBDPS_E_INVALID, "rho_s must be > 0");
  if (!(is_fin(p->d_p) && p->d_p >= 0.02 && p->d_p < 1.0)) return fail(LBDPS_E_INVALID, "d_p must be in [0.02, 1)");
  if (!(p->e_pp >= 0 && p->e_pp <= 1)) return fail(LBDPS_E_INVALID, "e_pp must be in [0, 1]");
  if (!(p->e_pw >= 0 && p->e_pw <= 1)) return fail(LBDPS_E_INVALID, "e_pw must be in [0, 1]");
  for (int a = 0; a < 2; ++a)
    if (!is_fin(p->g[a]) || !is_fin(p->body_force[a])) return fail(LBDPS_E_INVALID, "g and body_force must be finite");
  if (p->drag_ratio_mode < 0 || p->drag_ratio_mode > 2)
    return fail(LBDPS_E_INVALID, "drag_ratio_mode must be 0, 1 or 2");
  if (p->u_gas_porosity < 0 || p->u_gas_porosity > 2) return fail(LBDPS_E_INVALID, "u_gas_porosity must be 0..2");
  if (p->omega_mode < 0 || p->omega_mode > 1) return fail(LBDPS_E_INVALID, "omega_mode must be 0 or 1");
  if (p->pressure_force_sign < -1 || p->pressure_force_sign > 1)
    return fail(LBDPS_E_INVALID, "pressure_force_sign must be -1, 0 or 1");
  if (!is_fin(p->omega_dense)) return fail(LBDPS_E_INVALID, "omega_dense must be finite");
  if (!is_fin(p->cs_smag) || p->cs_smag < 0) return fail(LBDPS_E_INVALID, "cs_smag must be >= 0");
  if (p->particles_periodic_y < 0 || p->particles_periodic_y > 1)
    return fail(LBDPS_E_INVALID, "particles_periodic_y must be 0 or 1");
  if (p->diag_every < 0) return fail(LBDPS_E_INVALID, "diag_every must be >= 0");
  if (p->n_sub < 0 || p->n_sub > LBDPS_MAX_SUBSTEPS)
    return fail(LBDPS_E_INVALID, "n_sub must be in [0, " + std::to_string(LBDPS_MAX_SUBSTEPS) + "]");
  if (p->precision < 0 || p->precision > 3) return fail(LBDPS_E_INVALID, "precision must be 0..3");
  if (p->diagnostics < 0 || p->diagnostics > 1) return fail(LBDPS_E_INVALID, "diagnostics must be 0 or 1");
  // below 2^29: every per-particle and per-cell array is addressed by 32-bit byte offsets
  if (max_particles < 0 || max_particles >= (1ll << 29))
    return fail(LBDPS_E_SHAPE, "max_particles must be in [0, 2^29)");
  return LBDPS_OK;
}

lbdps_status lbdps_workspace_bytes(const lbdps_params *p, int64_t max_particles, size_t *bytes) {
  lbdps_status st = lbdps_validate_params(p, max_particles);
  if (st != LBDPS_OK) return st;
  if (!bytes) return fail(LBDPS_E_INVALID, "bytes is NULL");
  *bytes = carve(*p, max_particles, nullptr, nullptr);
  return LBDPS_OK;
}

lbdps_status lbdps_create(const lbdps_params *p, int64_t max_particles, void *d_workspace, size_t bytes,
                          const double *h_inlet_uy, void *stream, lbdps_ctx **out) {
  if (!out) return fail(LBDPS_E_INVALID, "out is NULL");
  *out = nullptr;
  lbdps_status st = lbdps_validate_params(p, max_particles);
  if (st != LBDPS_OK) return st;
  const size_t need = carve(*p, max_particles, nullptr, nullptr);
  if (!d_workspace) return fail(LBDPS_E_INVALID, "workspace is NULL");
  if (bytes < need) return fail(LBDPS_E_SHAPE, "workspace too small: need " + std::to_string(need) + " bytes");
  if (((uintptr_t)d_workspace & 255) != 0) return fail(LBDPS_E_INVALID, "workspace must be 256-byte aligned");
  lbdps_ctx *x = new (std::nothrow) lbdps_ctx();
  if (!x) return fail(LBDPS_E_DEVICE, "host allocation failed");
  x->p = *p;
  x->prec = p->precision;
  x->nx = p->nx;
  x->ny = p->ny;
  x->C = p->nx * p->ny;
  x->nmax = max_particles;
  x->nlut = lut_rows(p->d_p);
  x->stream = (hipStream_t)stream;
  x->dc = make_dconsts(*p);
  if ((st = check_hip(hipGetDevice(&x->device), "lbdps_create")) != LBDPS_OK ||
      (st = scratch_address(x->device, &x->scratch)) != LBDPS_OK) {
    delete x;
    return st;
  }
  carve(*p, max_particles, (char *)d_workspace, x);

  // per-count table and inlet profile, converted to the arithmetic type
  std::vector<double> lut = build_lut(*p);
  std::vector<double> inl(p->nx, 0.0);
  if (h_inlet_uy)
    for (int i = 0; i < p->nx; ++i) inl[i] = h_inlet_uy[i];
  auto upload = [&](void *dst, const std::vector<double> &v) -> lbdps_status {
    if (x->prec == PREC_FP64) return check_hip(hipMemcpy(dst, v.data(), v.size() * 8, hipMemcpyHostToDevice), "upload");
    std::vector<float> f(v.begin(), v.end());
    return check_hip(hipMemcpy(dst, f.data(), f.size() * 4, hipMemcpyHostToDevice), "upload");
  };
  std::vector<double> egv((size_t)x->nlut);
  for (int n = 0; n < x->nlut; ++n) egv[(size_t)n] = 1.0 - lut[(size_t)n * LUT_W + L_ES3];
  if ((st = upload(x->lut, lut)) != LBDPS_OK || (st = upload(x->inlet, inl)) != LBDPS_OK ||
      (st = check_hip(hipMemcpy(x->eg_tab, egv.data(), egv.size() * 8, hipMemcpyHostToDevice), "upload")) !=
          LBDPS_OK) {
    delete x;
    return st;
  }
  hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(x->C)), dim3(BLOCK), 0, x->stream, x->count, (long long)x->C, 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(BLOCK), 0, x->stream, x->flags, (long long)FLAG_COUNT, 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(BLOCK), 0, x->stream, x->need_sweep, 4ll, 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(x->nmax / RES_CHUNK + 1)), dim3(BLOCK), 0, x->stream, x->chunk_busy,
                     (long long)(x->nmax / RES_CHUNK + 1), 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(x->ntiles + 1)), dim3(BLOCK), 0, x->stream, x->tile_sum,
                     (long long)x->ntiles + 1, 0);
  st = dispatch(x, [&](auto impl) { return decltype(impl)::set_state(x, nullptr, nullptr, nullptr, 0); });
  if (st == LBDPS_OK) st = check_hip(hipStreamSynchronize(x->stream), "lbdps_create");
  if (st != LBDPS_OK) {
    delete x;
    return st;
  }
  *out = x;
  return LBDPS_OK;
}

lbdps_status lbdps_set_state(lbdps_ctx *x, const double *d_f, const double *d_pos, const double *d_vel, int64_t n) {
  if (!x) return fail(LBDPS_E_INVALID, "ctx is NULL");
  if (n < 0 || n > x->nmax) return fail(LBDPS_E_SHAPE, "n must be in [0, max_particles]");
  if (n > 0 && (!d_pos || !d_vel)) return fail(LBDPS_E_INVALID, "positions and velocities are required when n > 0");
  return dispatch(x, [&](auto impl) { return decltype(impl)::set_state(x, d_f, d_pos, d_vel, n); });
}

lbdps_status lbdps_step(lbdps_ctx *x, int32_t nsteps) {
  if (!x) return fail(LBDPS_E_INVALID, "ctx is NULL");
  if (nsteps < 0) return fail(LBDPS_E_INVALID, "nsteps must be >= 0");
  return dispatch(x, [&](auto impl) { return decltype(impl)::step(x, nsteps); });
}

lbdps_status lbdps_collide_particles(lbdps_ctx *x) {
  if (!x) return fail(LBDPS_E_INVALID, "ctx is NULL");
  return dispatch(x, [&](auto impl) { return decltype(impl)::collide_particles(x); });
}

lbdps_status lbdps3_bgk_step(const void *d_fin, void *d_fout, int32_t nx, int32_t ny, int32_t nz, double tau,
                             int32_t precision, void *stream) {
  if (!d_fin || !d_fout || d_fin == d_fout) return fail(LBDPS_E_INVALID, "d_fin and d_fout must be distinct buffers");
  if (nx < 1 || ny < 1 || nz < 1) return fail(LBDPS_E_SHAPE, "nx, ny and nz must be >= 1");
  if (!(std::isfinite(tau) && tau > 0.5)) return fail(LBDPS_E_INVALID, "tau must be > 0.5");
  const long long C = (long long)nx * ny * nz;
  const unsigned grid = (unsigned)((C + BLOCK - 1) / BLOCK);
  // 16-bit storage, even rows and 4-byte aligned buffers: two cells per thread
  const bool pairs = nx % 2 == 0 && ((uintptr_t)d_fin & 3) == 0 && ((uintptr_t)d_fout & 3) == 0;
  const unsigned grid2 = (unsigned)((C / 2 + BLOCK - 1) / BLOCK);
  const hipStream_t st = (hipStream_t)stream;
  switch (precision) {
    case PREC_FP64:
      hipLaunchKernelGGL(k3_bgk<PREC_FP64>, dim3(grid), dim3(BLOCK), 0, st, (const double *)d_fin, (double *)d_fout,
                         nx, ny, nz, tau);
      break;
    case PREC_FP32:
      hipLaunchKernelGGL(k3_bgk<PREC_FP32>, dim3(grid), dim3(BLOCK), 0, st, (const float *)d_fin, (float *)d_fout, nx,
                         ny, nz, (float)tau);
      break;
    case PREC_FP16DEV:
      if (pairs)
        hipLaunchKernelGGL(k3_bgk_pairs<PREC_FP16DEV>, dim3(grid2), dim3(BLOCK), 0, st, (const _Float16 *)d_fin,
                           (_Float16 *)d_fout, nx, ny, nz, (float)tau);
      else
        hipLaunchKernelGGL(k3_bgk<PREC_FP16DEV>, dim3(grid), dim3(BLOCK), 0, st, (const _Float16 *)d_fin,
                           (_Float16 *)d_fout, nx, ny, nz, (float)tau);
      break;
    case PREC_BF16DEV:
      if (pairs)
        hipLaunchKernelGGL(k3_bgk_pairs<PREC_BF16DEV>, dim3(grid2), dim3(BLOCK), 0, st, (const uint16_t *)d_fin,
                           (uint16_t *)d_fout, nx, ny, nz, (float)tau);
      else
        hipLaunchKernelGGL(k3_bgk<PREC_BF16DEV>, dim3(grid), dim3(BLOCK), 0, st, (const uint16_t *)d_fin,
                           (uint16_t *)d_fout, nx, ny, nz, (float)tau);
      break;
    default:
      return fail(LBDPS_E_INVALID, "precision must be 0..3");
  }
  return launch_status("lbdps3_bgk_step");
}

lbdps_status lbdps3_psm_step(const void *d_fin, void *d_fout, const int32_t *d_n, const void *d_vs, void *d_force,
                             int32_t nx, int32_t ny, int32_t nz, double tau, double d, int32_t precision,
                             void *stream) {
  if (!d_fin || !d_fout || d_fin == d_fout) return fail(LBDPS_E_INVALID, "d_fin and d_fout must be distinct buffers");
  if (!d_n || !d_vs || !d_force) return fail(LBDPS_E_INVALID, "d_n, d_vs and d_force must be device buffers");
  if (nx < 1 || ny < 1 || nz < 1) return fail(LBDPS_E_SHAPE, "nx, ny and nz must be >= 1");
  if (!(std::isfinite(tau) && tau > 0.5)) return fail(LBDPS_E_INVALID, "tau must be > 0.5");
  if (!(std::isfinite(d) && d > 0.0)) return fail(LBDPS_E_INVALID, "d must be > 0");
  const long long C = (long long)nx * ny * nz;
  const unsigned grid = (unsigned)((C + BLOCK - 1) / BLOCK);
  const double vol = M_PI * d * d * d / 6.0;          // sphere volume in cells
  const double cap = M_PI / (3.0 * std::sqrt(2.0));  // densest sphere packing
  // 16-bit storage, even rows, 4-byte aligned populations and 8-byte aligned
  // solids: two cells per thread
  const bool pairs = nx % 2 == 0 && ((uintptr_t)d_fin & 3) == 0 && ((uintptr_t)d_fout & 3) == 0 &&
                     ((uintptr_t)d_n & 7) == 0 && ((uintptr_t)d_vs & 7) == 0 && ((uintptr_t)d_force & 7) == 0;
  const unsigned grid2 = (unsigned)((C / 2 + BLOCK - 1) / BLOCK);
  const hipStream_t st = (hipStream_t)stream;
  switch (precision) {
    case PREC_FP64:
      hipLaunchKernelGGL(k3_psm<PREC_FP64>, dim3(grid), dim3(BLOCK), 0, st, (const double *)d_fin, (double *)d_fout,
                         d_n, (const double *)d_vs, (double *)d_force, nx, ny, nz, tau, vol, cap);
      break;
    case PREC_FP32:
      hipLaunchKernelGGL(k3_psm<PREC_FP32>, dim3(grid), dim3(BLOCK), 0, st, (const float *)d_fin, (float *)d_fout, d_n,
                         (const float *)d_vs, (float *)d_force, nx, ny, nz, (float)tau, (float)vol, (float)cap);
      break;
    case PREC_FP16DEV:
      if (pairs)
        hipLaunchKernelGGL(k3_psm_pairs<PREC_FP16DEV>, dim3(grid2), dim3(BLOCK), 0, st, (const _Float16 *)d_fin,
                           (_Float16 *)d_fout, nx, ny, nz, (float)tau, d_n, (const float *)d_vs, (float *)d_force,
                           (float)vol, (float)cap);
      else
        hipLaunchKernelGGL(k3_psm<PREC_FP16DEV>, dim3(grid), dim3(BLOCK), 0, st, (const _Float16 *)d_fin,
                           (_Float16 *)d_fout, d_n, (const float *)d_vs, (float *)d_force, nx, ny, nz, (float)tau,
                           (float)vol, (float)cap);
      break;
    case PREC_BF16DEV:
      if (pairs)
        hipLaunchKernelGGL(k3_psm_pairs<PREC_BF16DEV>, dim3(grid2), dim3(BLOCK), 0, st, (const uint16_t *)d_fin,
                           (uint16_t *)d_fout, nx, ny, nz, (float)tau, d_n, (const float *)d_vs, (float *)d_force,
                           (float)vol, (float)cap);
      else
        hipLaunchKernelGGL(k3_psm<PREC_BF16DEV>, dim3(grid), dim3(BLOCK), 0, st, (const uint16_t *)d_fin,
                           (uint16_t *)d_fout, d_n, (const float *)d_vs, (float *)d_force, nx, ny, nz, (float)tau,
                           (float)vol, (float)cap);
      break;
    default:
      return fail(LBDPS_E_INVALID, "precision must be 0..3");
  }
  return launch_status("lbdps3_psm_step");
}

lbdps_status lbdps_set_inlet(lbdps_ctx *x, const double *h_inlet_uy) {
  if (!x || !h_inlet_uy) return fail(LBDPS_E_INVALID, "ctx or inlet profile is NULL");
  for (int i = 0; i < x->nx; ++i)
    if (!is_fin(h_inlet_uy[i])) return fail(LBDPS_E_INVALID, "inlet velocities must be finite");
  lbdps_status st = check_hip(hipStreamSynchronize(x->stream), "lbdps_set_inlet");
  if (st != LBDPS_OK) return st;
  if (x->prec == PREC_FP64)
    return check_hip(hipMemcpy(x->inlet, h_inlet_uy, (size_t)x->nx * 8, hipMemcpyHostToDevice), "lbdps_set_inlet");
  std::vector<float> f(h_inlet_uy, h_inlet_uy + x->nx);
  return check_hip(hipMemcpy(x->inlet, f.data(), f.size() * 4, hipMemcpyHostToDevice), "lbdps_set_inlet");
}

lbdps_status lbdps_voidage(lbdps_ctx *x, int32_t y0, int32_t y1, double threshold, double *d_row_sum,
                           double *d_col_sum, int64_t *d_count) {
  if (!x) return fail(LBDPS_E_INVALID, "ctx is NULL");
  if (y0 < 0 || y1 > x->ny || y0 > y1) return fail(LBDPS_E_INVALID, "rows must satisfy 0 <= y0 <= y1 <= ny");
  if (!is_fin(threshold)) return fail(LBDPS_E_INVALID, "threshold must be finite");
  return dispatch(x, [&](auto impl) { return decltype(impl)::voidage(x, y0, y1, threshold, d_row_sum, d_col_sum,
                                                                     d_count); });
}

lbdps_status lbdps_count_histogram(lbdps_ctx *x, int64_t *h_hist, int32_t nbins) {
  if (!x || !h_hist) return fail(LBDPS_E_INVALID, "ctx or hist is NULL");
  if (nbins < 2 || nbins > HIST_BINS_MAX)
    return fail(LBDPS_E_INVALID, "nbins must be in [2, " + std::to_string(HIST_BINS_MAX) + "]");
  lbdps_status st = dispatch(x, [&](auto impl) { return decltype(impl)::count_histogram(x, nbins); });
  if (st != LBDPS_OK) return st;
  st = check_hip(hipMemcpyAsync(h_hist, x->hist, (size_t)nbins * 8, hipMemcpyDeviceToHost, x->stream),
                 "lbdps_count_histogram");
  if (st != LBDPS_OK) return st;
  return sync_and_check(x, "lbdps_count_histogram");
}

lbdps_status lbdps_get_fields(lbdps_ctx *x, double *d_rho, double *d_ugas, double *d_fpg, double *d_beta,
                              int32_t *d_ncell, double *d_vs) {
  if (!x) return fail(LBDPS_E_INVALID, "ctx is NULL");
  if ((d_ncell || d_vs) && !x->p.diagnostics) return fail(LBDPS_E_INVALID, "n_tot and v_s need diagnostics on");
  lbdps_status st = dispatch(x, [&](auto impl) {
    using I = decltype(impl);
    if (d_rho) I::get_field2(x, x->fld[0], nullptr, d_rho, x->prec == PREC_FP64 ? 0.0 : 1.0);
    if (d_ugas) I::get_field2(x, x->fld[1], x->fld[2], d_ugas);
    if (d_fpg) I::get_field2(x, x->fld[4], x->fld[5], d_fpg);
    if (d_beta) I::get_field2(x, x->fld[3], nullptr, d_beta);
    if (d_vs) I::get_field2(x, x->dg_vsx, x->dg_vsy, d_vs);
    return launch_status("lbdps_get_fields");
  });
  if (st != LBDPS_OK) return st;
  if (d_ncell) {
    st = check_hip(hipMemcpyAsync(d_ncell, x->dg_n, (size_t)x->C * 4, hipMemcpyDeviceToDevice, x->stream),
                   "lbdps_get_fields");
    if (st != LBDPS_OK) return st;
  }
  return sync_and_check(x, "lbdps_get_fields");
}

lbdps_status lbdps_get_particles(lbdps_ctx *x, double *d_pos, double *d_vel, double *d_fd, int32_t *d_cell) {
  if (!x) return fail(LBDPS_E_INVALID, "ctx is NULL");
  if (d_fd && !x->p.diagnostics) return fail(LBDPS_E_INVALID, "drag output needs diagnostics on");
  lbdps_status st = dispatch(x, [&](auto impl) {
    decltype(impl)::get_particles(x, d_pos, d_vel, d_fd, d_cell);
    return launch_status("lbdps_get_particles");
  });
  if (st != LBDPS_OK) return st;
  return sync_and_check(x, "lbdps_get_particles");
}

lbdps_status lbdps_get_accel(lbdps_ctx *x, double *d_acc) {
  if (!x || !d_acc) return fail(LBDPS_E_INVALID, "ctx or d_acc is NULL");
  if (!x->acx) return fail(LBDPS_E_INVALID, "the acceleration is held only with diagnostics on or n_sub > 1");
  if (x->n > 0) {
    lbdps_status st = dispatch(x, [&](auto impl) {
      using T = typename decltype(impl)::T;
      hipLaunchKernelGGL(k_get_field<T>, dim3(nblocks(x->n)), dim3(BLOCK), 0, x->stream, (const T *)x->acx,
                         (const T *)x->acy, (int)x->n, d_acc, 0.0);
      return launch_status("lbdps_get_accel");
    });
    if (st != LBDPS_OK) return st;
  }
  return sync_and_check(x, "lbdps_get_accel");
}

lbdps_status lbdps_get_pairs(lbdps_ctx *x, int32_t *d_pairs, int64_t cap, int64_t *n_out) {
  if (!x || !n_out) return fail(LBDPS_E_INVALID, "ctx or n_out is NULL");
  if (cap < 0 || (cap > 0 && !d_pairs)) return fail(LBDPS_E_INVALID, "bad pair buffer");
  const int N = (int)x->n;
  *n_out = 0;
  if (N == 0) return sync_and_check(x, "lbdps_get_pairs");
  dispatch(x, [&](auto impl) {
    decltype(impl)::rows(x);
    return LBDPS_OK;
  });
  // rank and perm are free between steps: counts, then offsets
  hipLaunchKernelGGL(k_pairs_count, dim3(nblocks(N)), dim3(BLOCK), 0, x->stream, x->slot, x->adj(), x->deg, N, x->rank);
  dispatch(x, [&](auto impl) {
    decltype(impl)::scan(x, x->rank, N, x->perm, 0);
    return LBDPS_OK;
  });
  hipLaunchKernelGGL(k_pairs_write, dim3(nblocks(N)), dim3(BLOCK), 0, x->stream, x->slot, x->adj(), x->deg, N, x->perm,
                     d_pairs, (long long)cap);
  lbdps_status st = launch_status("lbdps_get_pairs");
  if (st != LBDPS_OK) return st;
  int32_t total = 0;
  st = check_hip(hipMemcpyAsync(&total, x->perm + N, 4, hipMemcpyDeviceToHost, x->stream), "lbdps_get_pairs");
  if (st != LBDPS_OK) return st;
  st = sync_and_check(x, "lbdps_get_pairs");
  *n_out = total;
  return st;
}

lbdps_status lbdps_get_state(lbdps_ctx *x, double *d_f, double *d_pos, double *d_vel, int64_t *h_step) {
  if (!x) return fail(LBDPS_E_INVALID, "ctx is NULL");
  lbdps_status st = dispatch(x, [&](auto impl) {
    using I = decltype(impl);
    if (d_f) I::get_f(x, d_f);
    I::get_particles(x, d_pos, d_vel, nullptr, nullptr);
    return launch_status("lbdps_get_state");
  });
  if (st != LBDPS_OK) return st;
  if (h_step) *h_step = x->step;
  return sync_and_check(x, "lbdps_get_state");
}

// The conservation sums into the given scratch, copied to h_out.
lbdps_status conservation_with(lbdps_ctx *x, double *pc, double *pp, double *out, int32_t *flag, double h_out[6],
                               const char *what) {
  lbdps_status st = dispatch(x, [&](auto impl) {
    decltype(impl)::conservation(x, pc, pp, out, flag);
    return launch_status(what);
  });
  if (st != LBDPS_OK) return st;
  st = check_hip(hipMemcpyAsync(h_out, out, 6 * sizeof(double), hipMemcpyDeviceToHost, x->stream), what);
  if (st != LBDPS_OK) return st;
  st = sync_and_check(x, what);
  if (st != LBDPS_OK) return st;
  if (h_out[5] != 0.0) return fail(LBDPS_E_NONFINITE, "non-finite value in populations or velocities");
  return LBDPS_OK;
}

lbdps_status lbdps_conservation(lbdps_ctx *x, double h_out[6]) {
  if (!x || !h_out) return fail(LBDPS_E_INVALID, "ctx or out is NULL");
  return conservation_with(x, x->cons_pc, x->cons_pp, x->cons_out, x->nonfinite, h_out, "lbdps_conservation");
}

lbdps_status lbdps_diag_last(lbdps_ctx *x, double h_out[6], int64_t *h_step) {
  if (!x || !h_out || !h_step) return fail(LBDPS_E_INVALID, "ctx, out or step is NULL");
  lbdps_status st = sync_and_check(x, "lbdps_diag_last");
  if (st != LBDPS_OK) return st;
  *h_step = x->diag_step;
  for (int i = 0; i < 6; ++i) h_out[i] = 0.0;
  if (x->diag_step < 0) return LBDPS_OK;
  return check_hip(hipMemcpy(h_out, x->diag_out, 6 * sizeof(double), hipMemcpyDeviceToHost), "lbdps_diag_last");
}

lbdps_status lbdps_conservation_noalloc(lbdps_ctx *x, double h_out[6]) {
  if (!x || !h_out) return fail(LBDPS_E_INVALID, "ctx or out is NULL");
  static_assert(NOALLOC_FLAG * sizeof(double) + sizeof(int32_t) <= NOALLOC_SCRATCH_BYTES,
                "the conservation scratch fits the static array");
  if (!x->scratch) return fail(LBDPS_E_DEVICE, "no scratch address for the context's device");
  double *base = (double *)x->scratch;
  return conservation_with(x, base + NOALLOC_PC, base + NOALLOC_PP, base + NOALLOC_OUT,
                           (int32_t *)(base + NOALLOC_FLAG), h_out, "lbdps_conservation_noalloc");
}

lbdps_status lbdps_outlet_crossings(lbdps_ctx *x, int64_t *h_net, int64_t *h_steps) {
  if (!x || !h_net || !h_steps) return fail(LBDPS_E_INVALID, "ctx, h_net or h_steps is NULL");
  lbdps_status st = sync_and_check(x, "lbdps_outlet_crossings");
  if (st != LBDPS_OK) return st;
  unsigned long long total = 0;
  st = check_hip(hipMemcpy(&total, x->cross, sizeof(total), hipMemcpyDeviceToHost), "lbdps_outlet_crossings");
  if (st != LBDPS_OK) return st;
  *h_net = (int64_t)(total - x->cross_seen);  // modular difference of the running count
  *h_steps = x->step - x->cross_step0;
  x->cross_seen = total;
  x->cross_step0 = x->step;
  return LBDPS_OK;
}

lbdps_status lbdps_counters(lbdps_ctx *x, int64_t h_out[4]) {
  if (!x || !h_out) return fail(LBDPS_E_INVALID, "ctx or out is NULL");
  lbdps_status st = sync_and_check(x, "lbdps_counters");
  if (st != LBDPS_OK) return st;
  const int nbN = nblocks(x->n), nbC = x->drag_blocks;
  std::vector<long long> buf((size_t)std::max(nbN, nbC) + 1);
  // contacts: one partial per workgroup of the contact kernel; collisions and
  // wall hits of the resolution kernel: one per workgroup of that kernel
  long long *src[6] = {x->pair_part, x->coll_part, x->wall_part, x->wall0_part, x->collc_part, x->wallc_part};
  const int dst[6] = {0, 1, 2, 2, 1, 2};
  const int nres = Impl<PREC_FP32>::resolve_blocks(x);
  const int ncl = x->cluster_groups();
  const int len[6] = {nbN, nres, nres, nbN, ncl, ncl};
  for (int j = 0; j < 4; ++j) h_out[j] = 0;
  if (x->n > 0)
    for (int j = 0; j < 6; ++j) {
      if (x->sphere_tiles > 0 && (j == 0 || j == 3)) continue;  // the tile kernel counts these
      st = check_hip(hipMemcpy(buf.data(), src[j], (size_t)len[j] * 8, hipMemcpyDeviceToHost), "lbdps_counters");
      if (st != LBDPS_OK) return st;
      for (int b = 0; b < len[j]; ++b) h_out[dst[j]] += buf[b];
    }
  // the tile kernel's pairs, collisions and wall hits of the particles it resolved
  const int nst = x->n > 0 ? x->sphere_tiles : 0;
  if (nst > 0) {
    buf.resize((size_t)3 * nst);
    st = check_hip(hipMemcpy(buf.data(), x->tile_part, (size_t)3 * nst * 8, hipMemcpyDeviceToHost), "lbdps_counters");
    if (st != LBDPS_OK) return st;
    for (int j = 0; j < 3; ++j)
      for (int b = 0; b < nst; ++b) h_out[j] += buf[(size_t)j * nst + b];
  }
  if (x->p.diagnostics && x->n > 0) {
    st = check_hip(hipMemcpy(buf.data(), x->zero_part, (size_t)nbC * 8, hipMemcpyDeviceToHost), "lbdps_counters");
    if (st != LBDPS_OK) return st;
    for (int b = 0; b < nbC; ++b) h_out[3] += buf[b];
  }
  return LBDPS_OK;
}

lbdps_status lbdps_tile_stats(lbdps_ctx *x, int64_t h_out[2]) {
  if (!x || !h_out) return fail(LBDPS_E_INVALID, "ctx or out is NULL");
  lbdps_status st = sync_and_check(x, "lbdps_tile_stats");
  if (st != LBDPS_OK) return st;
  h_out[0] = 0;
  h_out[1] = 0;
  const int nst = x->n > 0 ? x->sphere_tiles : 0;
  if (nst == 0) {
    h_out[1] = x->n;
    return LBDPS_OK;
  }
  std::vector<long long> buf((size_t)nst);
  st = check_hip(hipMemcpy(buf.data(), x->tile_part + (size_t)3 * nst, (size_t)nst * 8, hipMemcpyDeviceToHost),
                 "lbdps_tile_stats");
  if (st != LBDPS_OK) return st;
  for (long long v : buf) h_out[1] += v;
  h_out[0] = x->n - h_out[1];
  return LBDPS_OK;
}

lbdps_status lbdps_time_kernels(lbdps_ctx *x, uint32_t mask) {
  if (!x) return fail(LBDPS_E_INVALID, "ctx is NULL");
  if (mask >> LBDPS_K_COUNT) return fail(LBDPS_E_INVALID, "unknown kernel bit in mask");
  x->timed = mask;
  return LBDPS_OK;
}

lbdps_status lbdps_kernel_times(lbdps_ctx *x, double *h_ms, int64_t *h_launches) {
  if (!x) return fail(LBDPS_E_INVALID, "ctx is NULL");
  lbdps_status st = check_hip(hipStreamSynchronize(x->stream), "lbdps_kernel_times");
  if (st != LBDPS_OK) return st;
  double ms[LBDPS_K_COUNT] = {0};
  long long cnt[LBDPS_K_COUNT] = {0};
  for (size_t i = 0; i < x->nmarks; ++i) {
    float t = 0.f;
    st = check_hip(hipEventElapsedTime(&t, x->marks[i].a, x->marks[i].b), "lbdps_kernel_times");
    if (st != LBDPS_OK) return st;
    ms[x->marks[i].k] += t;
    cnt[x->marks[i].k] += x->marks[i].extra ? 0 : 1;
  }
  x->nmarks = 0;
  for (int k = 0; k < LBDPS_K_COUNT; ++k) {
    if (h_ms) h_ms[k] = ms[k];
    if (h_launches) h_launches[k] = cnt[k];
  }
  return LBDPS_OK;
}

lbdps_status lbdps_set_tuning(lbdps_ctx *x, const lbdps_tuning *t) {
  if (!x || !t) return fail(LBDPS_E_INVALID, "ctx or tuning is NULL");
  if (t->cluster_lists < 1 || t->cluster_lists > BLOCK)
    return fail(LBDPS_E_INVALID, "cluster_lists must be in [1, 256]");
  if (t->cluster_groups_max < 1) return fail(LBDPS_E_INVALID, "cluster_groups_max must be >= 1");
  if (t->drag_tile < 0 || t->drag_tile >= DRAG_TILES)
    return fail(LBDPS_E_INVALID, "drag_tile must be 0 (32x8), 1 (64x4) or 2 (128x2)");
  if (t->sphere_tile < 0 || t->sphere_tile >= SPHERE_TILES)
    return fail(LBDPS_E_INVALID, "sphere_tile must be 0 (none), 1 (32x8), 2 (16x16) or 3 (64x4)");
  x->tune = *t;
  return LBDPS_OK;
}

}  // extern "C"

namespace {

// Launch shapes the autotuner tries (all give identical results).
const lbdps_tuning kTuneCandidates[] = {
    {1, RC_GROUPS_MAX, 0}, {2, RC_GROUPS_MAX, 0}, {4, RC_GROUPS_MAX, 0}, {8, RC_GROUPS_MAX, 0},
    {16, RC_GROUPS_MAX, 0}, {1, 4096, 0},         {1, 1024, 0},          {4, 1024, 0},
    {1, 128, 0},  // few contacts: a small grid reads the candidate counts and is done
};
constexpr int kTuneN = (int)(sizeof(kTuneCandidates) / sizeof(kTuneCandidates[0]));

// Milliseconds of the work fn enqueues on stream st.
template <class F> lbdps_status time_on(hipStream_t st, F &&fn, float *ms) {
  hipEvent_t a = nullptr, b = nullptr;
  lbdps_status r = check_hip(hipEventCreate(&a), "autotune");
  if (r == LBDPS_OK) r = check_hip(hipEventCreate(&b), "autotune");
  if (r == LBDPS_OK) r = check_hip(hipEventRecord(a, st), "autotune");
  if (r == LBDPS_OK) r = fn();
  if (r == LBDPS_OK) r = check_hip(hipEventRecord(b, st), "autotune");
  if (r == LBDPS_OK) r = check_hip(hipEventSynchronize(b), "autotune");
  if (r == LBDPS_OK) r = check_hip(hipEventElapsedTime(ms, a, b), "autotune");
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  return r;
}

// Size class of a bed: particle counts 1..2048 -> 0, ..4096 -> 1, ...; none -> -1.
int size_class(long long n) {
  if (n <= 0) return -1;
  int c = 0;
  while ((2048ll << c) < n) ++c;
  return c;
}

}  // namespace

extern "C" {

lbdps_status lbdps_autotune(lbdps_ctx *x, int32_t steps, lbdps_tuning *chosen) {
  if (!x) return fail(LBDPS_E_INVALID, "ctx is NULL");
  if (steps < 1) return fail(LBDPS_E_INVALID, "steps must be >= 1");
  // Two interleaved rounds over the candidates; each keeps its faster time, so
  // a single disturbed measurement does not decide.  The cluster-resolution
  // shapes first (under the context's drag tile), then the drag tile shapes
  // under the chosen cluster shape: the two phases do not share work.
  const lbdps_tuning start = x->tune;
  constexpr int NC = SPHERE_TILES + kTuneN + DRAG_TILES;
  float t[NC];
  lbdps_tuning cand[NC];
  auto run = [&](int c0, int c1) -> lbdps_status {
    for (int round = 0; round < 2; ++round)
      for (int c = c0; c < c1; ++c) {
        x->tune = cand[c];
        float ms = 0.f;
        lbdps_status st = time_on(
            x->stream, [&]() { return dispatch(x, [&](auto impl) { return decltype(impl)::step(x, steps); }); },
            &ms);
        if (st != LBDPS_OK) return st;
        t[c] = round == 0 ? ms : std::min(t[c], ms);
      }
    int bc = c0;
    for (int c = c0 + 1; c < c1; ++c)
      if (t[c] < t[bc]) bc = c;
    x->tune = cand[bc];
    return LBDPS_OK;
  };
  // the collision stage's tile shapes (none among them), then the cluster
  // shapes, then the drag tiles, each under the choices before it
  for (int c = 0; c < SPHERE_TILES; ++c) {
    cand[c] = start;
    cand[c].sphere_tile = c;
  }
  lbdps_status st = run(0, SPHERE_TILES);
  if (st == LBDPS_OK) {
    for (int c = 0; c < kTuneN; ++c) {
      cand[SPHERE_TILES + c] = kTuneCandidates[c];
      cand[SPHERE_TILES + c].drag_tile = x->tune.drag_tile;
      cand[SPHERE_TILES + c].sphere_tile = x->tune.sphere_tile;
    }
    st = run(SPHERE_TILES, SPHERE_TILES + kTuneN);
  }
  if (st == LBDPS_OK) {
    for (int d = 0; d < DRAG_TILES; ++d) {
      cand[SPHERE_TILES + kTuneN + d] = x->tune;
      cand[SPHERE_TILES + kTuneN + d].drag_tile = d;
    }
    st = run(SPHERE_TILES + kTuneN, NC);
  }
  if (st != LBDPS_OK) {
    x->tune = start;
    return st;
  }
  if (chosen) *chosen = x->tune;
  return sync_and_check(x, "lbdps_autotune");
}

lbdps_status lbdps_get_tuning(lbdps_ctx *x, lbdps_tuning *t) {
  if (!x || !t) return fail(LBDPS_E_INVALID, "ctx or tuning is NULL");
  *t = x->tune;
  return LBDPS_OK;
}

lbdps_status lbdps_destroy(lbdps_ctx *x) {
  if (!x) return fail(LBDPS_E_INVALID, "ctx is NULL");
  if (x->in_batch) return fail(LBDPS_E_INVALID, "a bed of a batch is destroyed with the batch");
  delete x;
  return LBDPS_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batches of beds
struct lbdps_batch {
  int nbeds = 0, prec = 0;
  std::vector<lbdps_ctx *> beds;
  hipStream_t stream = nullptr;
  // two device tables (eager stepping, captured graph), each: BedArgs[nbeds], then off[PH_COUNT][nbeds + 1]
  char *d_tab[2]{};
  size_t tab_bytes = 0, args_bytes = 0;
  char *h_tab = nullptr;  // pinned staging copy of a table
  hipEvent_t tab_done = nullptr;
  bool tab_inflight = false;
  int total[2][PH_COUNT]{};
  int tile[2]{};  // drag tile shape each table was written for
  // bed state the graph's table describes
  std::vector<int> snap_cf, snap_cp;
  std::vector<long long> snap_n;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_steps = 0;
  // per-kernel event timing of eager batched steps
  uint32_t timed = 0;
  std::vector<lbdps_ctx::Mark> marks;
  size_t nmarks = 0;
  ~lbdps_batch() {
    for (auto &m : marks) {
      (void)hipEventDestroy(m.a);
      (void)hipEventDestroy(m.b);
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (tab_done) (void)hipEventDestroy(tab_done);
    if (h_tab) (void)hipHostFree(h_tab);
    for (auto *b : beds) delete b;
  }
};

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

template <int P> struct BatchImpl {
  using T = typename Prec<P>::T;
  using S = typename Prec<P>::S;
  using I = Impl<P>;

  static size_t args_bytes(int nbeds) { return align256((size_t)nbeds * sizeof(BedArgs<P>)); }
  static size_t table_bytes(int nbeds) { return args_bytes(nbeds) + align256((size_t)PH_COUNT * (nbeds + 1) * 4); }

  static BedArgs<P> args(const lbdps_ctx *x) {
    BedArgs<P> a{};
    a.k = I::consts(x);
    for (int b = 0; b < 2; ++b) {
      a.f[b] = (S *)x->f[b];
      a.key[b] = x->key[b];
      a.pid[b] = x->pid[b];
      a.px[b] = (T *)x->px[b];
      a.py[b] = (T *)x->py[b];
      a.vx[b] = (T *)x->vx[b];
      a.vy[b] = (T *)x->vy[b];
    }
    a.fl = I::fields(x);
    a.lut = (const T *)x->lut;
    a.inlet = (const T *)x->inlet;
    a.cs = x->cs;
    a.count = x->count;
    a.stay = x->stay;
    a.rank = x->rank;
    a.slot = x->slot;
    a.flags = x->flags;
    a.deg = x->deg;
    a.done = x->done;
    a.ticket = x->ticket;
    a.chunk_busy = x->chunk_busy;
    a.need_sweep = x->need_sweep;
    a.roots = x->roots;
    a.rcount = x->rcount;
    a.adj = x->adj();
    a.pair_part = x->pair_part;
    a.wall0_part = x->wall0_part;
    a.coll_part = x->coll_part;
    a.wall_part = x->wall_part;
    a.collc_part = x->collc_part;
    a.wallc_part = x->wallc_part;
    a.ts = I::tiles(x);
    a.cf = x->cf;
    a.cp = x->cp;
    a.cp_moves = x->n > 0;
    a.nlists = nblocks(x->n);
    return a;
  }

  // Workgroups of each phase for one bed, as the single-bed step launches
  // them; the drag under the batch's tile shape `tile`.
  static void blocks(const lbdps_ctx *x, int tile, int nb[PH_COUNT]) {
    for (int i = 0; i < PH_COUNT; ++i) nb[i] = 0;
    nb[PH_COLLIDE] = nblocks(x->C);
    if (x->n == 0) return;
    nb[PH_DRAG] = I::drag_tiles(x, tile);
    nb[PH_SCAN] = x->ntiles;
    nb[PH_SCATTER] = nblocks(x->n);
    nb[PH_CONTACTS] = nblocks(x->n);
    nb[PH_CLUSTERS] = x->cluster_groups();
    nb[PH_RESOLVE] = I::resolve_blocks(x);
  }

  // Fills table t (0 eager, 1 graph) from the beds' current state.
  static lbdps_status write_table(lbdps_batch *B, int t) {
    if (B->tab_inflight) {
      lbdps_status st = check_hip(hipEventSynchronize(B->tab_done), "batch table");
      if (st != LBDPS_OK) return st;
      B->tab_inflight = false;
    }
    BedArgs<P> *a = (BedArgs<P> *)B->h_tab;
    int *off = (int *)(B->h_tab + B->args_bytes);
    const int nb1 = B->nbeds + 1;
    for (int ph = 0; ph < PH_COUNT; ++ph) off[ph * nb1] = 0;
    // one drag tile shape for the whole launch: bed 0's (the batch autotuner
    // gives every bed the same)
    const int tile = B->beds[0]->tune.drag_tile;
    for (int b = 0; b < B->nbeds; ++b)
      if (B->beds[b]->tune.drag_tile != tile)
        return fail(LBDPS_E_INVALID, "the beds of a batch must share one drag tile shape");
    B->tile[t] = tile;
    for (int b = 0; b < B->nbeds; ++b) {
      const lbdps_ctx *x = B->beds[b];
      a[b] = args(x);
      int nb[PH_COUNT];
      blocks(x, tile, nb);
      for (int ph = 0; ph < PH_COUNT; ++ph) {
        const long long v = (long long)off[ph * nb1 + b] + nb[ph];
        if (v > 0x7fffffffll) return fail(LBDPS_E_SHAPE, "batch too large for one launch per phase");
        off[ph * nb1 + b + 1] = (int)v;
      }
    }
    for (int ph = 0; ph < PH_COUNT; ++ph) B->total[t][ph] = off[ph * nb1 + B->nbeds];
    lbdps_status st = check_hip(hipMemcpyAsync(B->d_tab[t], B->h_tab, B->tab_bytes, hipMemcpyHostToDevice, B->stream),
                                "batch table upload");
    if (st != LBDPS_OK) return st;
    st = check_hip(hipEventRecord(B->tab_done, B->stream), "batch table upload");
    B->tab_inflight = st == LBDPS_OK;
    return st;
  }

  // The step phase's kernel class (k as in lbdps_kernel).
  static int phase_kernel(int ph) {
    switch (ph) {
      case PH_COLLIDE: return LBDPS_K_COLLIDE;
      case PH_DRAG: return LBDPS_K_DRAG;
      case PH_SCAN: return LBDPS_K_SCAN;
      case PH_SCATTER: return LBDPS_K_SCATTER;
      case PH_CONTACTS: return LBDPS_K_CONTACTS;
      default: return LBDPS_K_RESOLVE;  // the cluster kernel and the ordered sweep
    }
  }
  // Events for a timed launch of kernel class k in an eager batched step,
  // stamped by the dispatch itself (the kernel's own time); false when k is
  // not timed.  extra: a further launch of the same class in the step.
  static bool bmark(lbdps_batch *B, int k, bool extra, hipEvent_t &a, hipEvent_t &b) {
    if (!(B->timed >> k & 1u)) return false;
    if (B->nmarks == B->marks.size()) {
      lbdps_ctx::Mark m{};
      if (hipEventCreate(&m.a) != hipSuccess || hipEventCreate(&m.b) != hipSuccess) return false;
      B->marks.push_back(m);
    }
    lbdps_ctx::Mark &m = B->marks[B->nmarks++];
    m.k = k;
    m.extra = extra;
    a = m.a;
    b = m.b;
    return true;
  }

  static void launch_steps(lbdps_batch *B, int t, int nsteps) {
    const BedArgs<P> *tab = (const BedArgs<P> *)B->d_tab[t];
    const int *off = (const int *)(B->d_tab[t] + B->args_bytes);
    const int nb1 = B->nbeds + 1, nbeds = B->nbeds;
    const int *tot = B->total[t];
    const bool timing = t == 0;  // never inside a captured graph
    for (int it = 0; it < nsteps; ++it) {
      const int flip = it & 1;
#define LBDPS_LAUNCH(kern, ph)                                                                                      \
  if (tot[ph] > 0) {                                                                                                \
    hipEvent_t ea = nullptr, eb = nullptr;                                                                          \
    if (timing && bmark(B, phase_kernel(ph), ph == PH_RESOLVE, ea, eb))                                             \
      hipExtLaunchKernelGGL(kern, dim3(tot[ph]), dim3(BLOCK), 0, B->stream, ea, eb, 0, tab, off + (ph) * nb1,       \
                            nbeds, flip);                                                                           \
    else                                                                                                            \
      hipLaunchKernelGGL(kern, dim3(tot[ph]), dim3(BLOCK), 0, B->stream, tab, off + (ph) * nb1, nbeds, flip);       \
  }
      LBDPS_LAUNCH(kb_collide<P>, PH_COLLIDE)
      const bool flat = drag_flat(tot[PH_DRAG]);
      switch (B->tile[t]) {
        case 1:
          if (flat) { LBDPS_LAUNCH((kb_drag_flat<P, 64>), PH_DRAG) } else { LBDPS_LAUNCH((kb_drag<P, 64>), PH_DRAG) }
          break;
        case 2:
          if (flat) { LBDPS_LAUNCH((kb_drag_flat<P, 128>), PH_DRAG) } else { LBDPS_LAUNCH((kb_drag<P, 128>), PH_DRAG) }
          break;
        default:
          if (flat) { LBDPS_LAUNCH((kb_drag_flat<P, 32>), PH_DRAG) } else { LBDPS_LAUNCH((kb_drag<P, 32>), PH_DRAG) }
      }
      LBDPS_LAUNCH(kb_scan<P>, PH_SCAN)
      LBDPS_LAUNCH(kb_scatter<P>, PH_SCATTER)
      LBDPS_LAUNCH(kb_contacts<P>, PH_CONTACTS)
      LBDPS_LAUNCH(kb_clusters<P>, PH_CLUSTERS)
      LBDPS_LAUNCH(kb_resolve<P>, PH_RESOLVE)
#undef LBDPS_LAUNCH
    }
  }

  static void advance(lbdps_batch *B, int nsteps) {
    for (auto *x : B->beds) {
      x->sphere_tiles = 0;  // the batched collision stage is the row path
      x->cf ^= nsteps & 1;
      if (x->n > 0) x->cp ^= nsteps & 1;
      x->step += nsteps;
    }
  }

  static void rebin_all(lbdps_batch *B) {
    for (auto *x : B->beds)
      if (!x->bins_valid) I::rebin(x);
  }

  static lbdps_status step(lbdps_batch *B, int nsteps) {
    if (nsteps == 0) return LBDPS_OK;
    rebin_all(B);
    lbdps_status st = write_table(B, 0);
    if (st != LBDPS_OK) return st;
    launch_steps(B, 0, nsteps);
    advance(B, nsteps);
    return launch_status("lbdps_batch_step");
  }

  static lbdps_status capture(lbdps_batch *B, int nsteps) {
    rebin_all(B);
    lbdps_status st = write_table(B, 1);
    if (st != LBDPS_OK) return st;
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    B->exec = nullptr;
    B->graph = nullptr;
    B->graph_steps = 0;
    st = check_hip(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal), "lbdps_batch_capture");
    if (st != LBDPS_OK) return st;
    launch_steps(B, 1, nsteps);
    hipGraph_t g = nullptr;
    st = check_hip(hipStreamEndCapture(B->stream, &g), "lbdps_batch_capture");
    if (st != LBDPS_OK) return st;
    B->graph = g;
    st = check_hip(hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0), "lbdps_batch_capture");
    if (st != LBDPS_OK) return st;
    B->graph_steps = nsteps;
    B->snap_cf.clear();
    B->snap_cp.clear();
    B->snap_n.clear();
    for (auto *x : B->beds) {
      B->snap_cf.push_back(x->cf);
      B->snap_cp.push_back(x->cp);
      B->snap_n.push_back(x->n);
    }
    return LBDPS_OK;
  }
};

template <class F> lbdps_status dispatch_batch(int prec, F &&fn) {
  switch (prec) {
    case PREC_FP64: return fn(BatchImpl<PREC_FP64>{});
    case PREC_FP32: return fn(BatchImpl<PREC_FP32>{});
    case PREC_FP16DEV: return fn(BatchImpl<PREC_FP16DEV>{});
    case PREC_BF16DEV: return fn(BatchImpl<PREC_BF16DEV>{});
  }
  return fail(LBDPS_E_INVALID, "unknown precision");
}

// Layout of a batch workspace: the two tables, then each bed's workspace.
lbdps_status batch_layout(const lbdps_params *beds, int32_t nbeds, const int64_t *max_particles, size_t *tab,
                          std::vector<size_t> *bed_off, size_t *total) {
  if (!beds || !max_particles) return fail(LBDPS_E_INVALID, "beds or max_particles is NULL");
  if (nbeds < 1) return fail(LBDPS_E_SHAPE, "nbeds must be >= 1");
  const int prec = beds[0].precision;
  for (int b = 0; b < nbeds; ++b) {
    lbdps_status st = lbdps_validate_params(&beds[b], max_particles[b]);
    if (st != LBDPS_OK) return fail(st, "bed " + std::to_string(b) + ": " + lbdps_last_error());
    if (beds[b].precision != prec) return fail(LBDPS_E_INVALID, "all beds of a batch share one precision");
    if (beds[b].diagnostics) return fail(LBDPS_E_UNSUPPORTED, "batched beds do not record diagnostics");
    if (n_sub_of(beds[b]) > 1) return fail(LBDPS_E_UNSUPPORTED, "batched beds take one particle sub-step");
    if (beds[b].diag_every > 0) return fail(LBDPS_E_UNSUPPORTED, "batched beds take no periodic check");
  }
  size_t tb = 0;
  lbdps_status st = dispatch_batch(prec, [&](auto impl) {
    tb = decltype(impl)::table_bytes(nbeds);
    return LBDPS_OK;
  });
  if (st != LBDPS_OK) return st;
  size_t off = 2 * tb;
  if (bed_off) bed_off->clear();
  for (int b = 0; b < nbeds; ++b) {
    if (bed_off) bed_off->push_back(off);
    off += align256(carve(beds[b], max_particles[b], nullptr, nullptr));
  }
  *tab = tb;
  *total = off;
  return LBDPS_OK;
}

}  // namespace

extern "C" {

lbdps_status lbdps_batch_workspace_bytes(const lbdps_params *beds, int32_t nbeds, const int64_t *max_particles,
                                         size_t *bytes) {
  if (!bytes) return fail(LBDPS_E_INVALID, "bytes is NULL");
  size_t tab = 0;
  return batch_layout(beds, nbeds, max_particles, &tab, nullptr, bytes);
}

lbdps_status lbdps_batch_create(const lbdps_params *beds, int32_t nbeds, const int64_t *max_particles,
                                const double *const *h_inlet_uy, void *d_workspace, size_t bytes, void *stream,
                                lbdps_batch **out) {
  if (!out) return fail(LBDPS_E_INVALID, "out is NULL");
  *out = nullptr;
  size_t tab = 0, total = 0;
  std::vector<size_t> bed_off;
  lbdps_status st = batch_layout(beds, nbeds, max_particles, &tab, &bed_off, &total);
  if (st != LBDPS_OK) return st;
  if (!d_workspace) return fail(LBDPS_E_INVALID, "workspace is NULL");
  if (bytes < total) return fail(LBDPS_E_SHAPE, "workspace too small: need " + std::to_string(total) + " bytes");
  if (((uintptr_t)d_workspace & 255) != 0) return fail(LBDPS_E_INVALID, "workspace must be 256-byte aligned");
  lbdps_batch *B = new (std::nothrow) lbdps_batch();
  if (!B) return fail(LBDPS_E_DEVICE, "host allocation failed");
  B->nbeds = nbeds;
  B->prec = beds[0].precision;
  B->stream = (hipStream_t)stream;
  B->tab_bytes = tab;
  dispatch_batch(B->prec, [&](auto impl) {
    B->args_bytes = decltype(impl)::args_bytes(nbeds);
    return LBDPS_OK;
  });
  B->d_tab[0] = (char *)d_workspace;
  B->d_tab[1] = (char *)d_workspace + tab;
  st = check_hip(hipHostMalloc((void **)&B->h_tab, tab, hipHostMallocDefault), "lbdps_batch_create");
  if (st == LBDPS_OK)
    st = check_hip(hipEventCreateWithFlags(&B->tab_done, hipEventDisableTiming), "lbdps_batch_create");
  for (int b = 0; st == LBDPS_OK && b < nbeds; ++b) {
    lbdps_ctx *x = nullptr;
    st = lbdps_create(&beds[b], max_particles[b], (char *)d_workspace + bed_off[b], total - bed_off[b],
                      h_inlet_uy ? h_inlet_uy[b] : nullptr, stream, &x);
    if (st == LBDPS_OK) {
      x->in_batch = true;
      B->beds.push_back(x);
    }
  }
  if (st != LBDPS_OK) {
    delete B;
    return st;
  }
  *out = B;
  return LBDPS_OK;
}

lbdps_status lbdps_batch_bed(lbdps_batch *B, int32_t bed, lbdps_ctx **out) {
  if (!B || !out) return fail(LBDPS_E_INVALID, "batch or out is NULL");
  if (bed < 0 || bed >= B->nbeds) return fail(LBDPS_E_SHAPE, "bed index out of range");
  *out = B->beds[bed];
  return LBDPS_OK;
}

lbdps_status lbdps_batch_step(lbdps_batch *B, int32_t nsteps) {
  if (!B) return fail(LBDPS_E_INVALID, "batch is NULL");
  if (nsteps < 0) return fail(LBDPS_E_INVALID, "nsteps must be >= 0");
  return dispatch_batch(B->prec, [&](auto impl) { return decltype(impl)::step(B, nsteps); });
}

lbdps_status lbdps_batch_capture(lbdps_batch *B, int32_t nsteps) {
  if (!B) return fail(LBDPS_E_INVALID, "batch is NULL");
  if (nsteps < 2 || (nsteps & 1)) return fail(LBDPS_E_INVALID, "nsteps must be even and >= 2");
  if (!B->stream) return fail(LBDPS_E_INVALID, "capture needs a stream other than the null stream");
  return dispatch_batch(B->prec, [&](auto impl) { return decltype(impl)::capture(B, nsteps); });
}

lbdps_status lbdps_batch_launch(lbdps_batch *B) {
  if (!B) return fail(LBDPS_E_INVALID, "batch is NULL");
  if (!B->exec) return fail(LBDPS_E_INVALID, "no captured graph");
  for (int b = 0; b < B->nbeds; ++b) {
    const lbdps_ctx *x = B->beds[b];
    if (!x->bins_valid || x->cf != B->snap_cf[b] || x->cp != B->snap_cp[b] || x->n != B->snap_n[b])
      return fail(LBDPS_E_INVALID, "bed " + std::to_string(b) + " changed since the capture; capture again");
  }
  lbdps_status st = check_hip(hipGraphLaunch(B->exec, B->stream), "lbdps_batch_launch");
  if (st != LBDPS_OK) return st;
  return dispatch_batch(B->prec, [&](auto impl) {
    decltype(impl)::advance(B, B->graph_steps);
    return LBDPS_OK;
  });
}

lbdps_status lbdps_batch_sync(lbdps_batch *B) {
  if (!B) return fail(LBDPS_E_INVALID, "batch is NULL");
  for (int b = 0; b < B->nbeds; ++b) {
    lbdps_status st = sync_and_check(B->beds[b], "lbdps_batch_sync");
    if (st != LBDPS_OK) return fail(st, "bed " + std::to_string(b) + ": " + lbdps_last_error());
  }
  return LBDPS_OK;
}

lbdps_status lbdps_batch_time_kernels(lbdps_batch *B, uint32_t mask) {
  if (!B) return fail(LBDPS_E_INVALID, "batch is NULL");
  if (mask >> LBDPS_K_COUNT) return fail(LBDPS_E_INVALID, "unknown kernel bit in mask");
  B->timed = mask;
  return LBDPS_OK;
}

lbdps_status lbdps_batch_kernel_times(lbdps_batch *B, double *h_ms, int64_t *h_launches) {
  if (!B) return fail(LBDPS_E_INVALID, "batch is NULL");
  lbdps_status st = check_hip(hipStreamSynchronize(B->stream), "lbdps_batch_kernel_times");
  if (st != LBDPS_OK) return st;
  double ms[LBDPS_K_COUNT] = {0};
  long long cnt[LBDPS_K_COUNT] = {0};
  for (size_t i = 0; i < B->nmarks; ++i) {
    float t = 0.f;
    st = check_hip(hipEventElapsedTime(&t, B->marks[i].a, B->marks[i].b), "lbdps_batch_kernel_times");
    if (st != LBDPS_OK) return st;
    ms[B->marks[i].k] += t;
    cnt[B->marks[i].k] += B->marks[i].extra ? 0 : 1;
  }
  B->nmarks = 0;
  for (int k = 0; k < LBDPS_K_COUNT; ++k) {
    if (h_ms) h_ms[k] = ms[k];
    if (h_launches) h_launches[k] = cnt[k];
  }
  return LBDPS_OK;
}

lbdps_status lbdps_batch_autotune(lbdps_batch *B, int32_t steps, const char *cache_path) {
  if (!B) return fail(LBDPS_E_INVALID, "batch is NULL");
  if (steps < 1) return fail(LBDPS_E_INVALID, "steps must be >= 1");
  std::map<int, std::vector<int>> cls;
  for (int b = 0; b < B->nbeds; ++b) cls[size_class(B->beds[b]->n)].push_back(b);
  cls.erase(-1);
  const std::string head = "lbdps-tune 2 precision " + std::to_string(B->prec);
  std::map<int, lbdps_tuning> cached;
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    if (in && std::getline(in, line) && line == head) {
      int c;
      lbdps_tuning t{};
      while (in >> c >> t.cluster_lists >> t.cluster_groups_max >> t.drag_tile) cached[c] = t;
    }
  }
  // The drag tile shape is one for the whole batch (one launch per phase):
  // the cached one, else bed 0's while the classes are tuned, then the
  // fastest of the shapes on the whole batched step.
  bool all_cached = true;
  for (auto &kv : cls) all_cached = all_cached && cached.count(kv.first);
  int tile = all_cached && !cached.empty() ? cached.begin()->second.drag_tile : B->beds[0]->tune.drag_tile;
  if (tile < 0 || tile >= DRAG_TILES) tile = 0;
  for (auto *x : B->beds) x->tune.drag_tile = tile;
  for (auto &kv : cls) {
    auto it = cached.find(kv.first);
    if (it != cached.end()) {
      for (int b : kv.second) {
        B->beds[b]->tune = it->second;
        B->beds[b]->tune.drag_tile = tile;
      }
      continue;
    }
    float t[kTuneN];
    for (int round = 0; round < 2; ++round)  // as lbdps_autotune: the faster of two times per candidate
      for (int c = 0; c < kTuneN; ++c) {
        for (int b : kv.second) {
          B->beds[b]->tune = kTuneCandidates[c];
          B->beds[b]->tune.drag_tile = tile;
        }
        float ms = 0.f;
        lbdps_status st = time_on(B->stream, [&]() { return lbdps_batch_step(B, steps); }, &ms);
        if (st != LBDPS_OK) return st;
        t[c] = round == 0 ? ms : std::min(t[c], ms);
      }
    int bc = 0;
    for (int c = 1; c < kTuneN; ++c)
      if (t[c] < t[bc]) bc = c;
    lbdps_tuning bt = kTuneCandidates[bc];
    bt.drag_tile = tile;
    for (int b : kv.second) B->beds[b]->tune = bt;
    cached[kv.first] = bt;
  }
  if (!all_cached) {
    float t[DRAG_TILES];
    for (int round = 0; round < 2; ++round)
      for (int d = 0; d < DRAG_TILES; ++d) {
        for (auto *x : B->beds) x->tune.drag_tile = d;
        float ms = 0.f;
        lbdps_status st = time_on(B->stream, [&]() { return lbdps_batch_step(B, steps); }, &ms);
        if (st != LBDPS_OK) return st;
        t[d] = round == 0 ? ms : std::min(t[d], ms);
      }
    tile = 0;
    for (int d = 1; d < DRAG_TILES; ++d)
      if (t[d] < t[tile]) tile = d;
    for (auto *x : B->beds) x->tune.drag_tile = tile;
    for (auto &kv : cached) kv.second.drag_tile = tile;
  }
  if (cache_path) {
    std::ofstream out(cache_path);
    if (!out) return fail(LBDPS_E_INVALID, std::string("cannot write the tuning cache ") + cache_path);
    out << head << "\n";
    for (auto &kv : cached)
      out << kv.first << " " << kv.second.cluster_lists << " " << kv.second.cluster_groups_max << " "
          << kv.second.drag_tile << "\n";
  }
  return lbdps_batch_sync(B);
}

lbdps_status lbdps_batch_destroy(lbdps_batch *B) {
  if (!B) return fail(LBDPS_E_INVALID, "batch is NULL");
  (void)hipStreamSynchronize(B->stream);
  for (auto *x : B->beds) x->in_batch = false;
  delete B;
  return LBDPS_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ the 3-D coupled step
struct lbdps3_ctx {
  lbdps3_params p{};
  int prec = 0, nx = 0, ny = 0, nz = 0, C = 0, nlut = 0;
  long long nmax = 0, n = 0;
  hipStream_t stream = nullptr;
  int cf = 0, cp = 0;
  bool bins_valid = false;
  long long step = 0;
  double dtau = 0, dd = 0, dmu = 0, dvp = 0, dm = 0, done_e = 0, dfp = 0, dgeff[3]{}, dhalfG[3]{}, dsrc[Q3]{};
  void *f[2]{};
  void *fld[10]{};  // rho, ugx, ugy, ugz, beta, es, fpx, fpy, fpz, the packed interpolation nodes [C][8]
  int32_t *key[2]{}, *pid[2]{};
  void *pos[2][3]{}, *vel[2][3]{};
  int32_t *count = nullptr, *cs = nullptr, *rank = nullptr, *slot = nullptr, *deg = nullptr, *done = nullptr;
  long long *adj_in = nullptr, *adj_ov = nullptr;
  int32_t *ticket = nullptr, *flags = nullptr, *chunk_busy = nullptr, *spart = nullptr, *pcnt = nullptr;
  long long *pair_part = nullptr, *coll_part = nullptr, *collc_part = nullptr;
  double *cons_pc = nullptr, *cons_pp = nullptr, *cons_out = nullptr;  // conservation scratch
  int32_t *cons_flag = nullptr;
  long long *roots = nullptr;  // candidate cluster roots, BLOCK per contact workgroup
  int32_t *rcount = nullptr, *need_sweep = nullptr;
  void *lut = nullptr;
  int32_t *dg_n = nullptr;
  void *dg_fd = nullptr, *dg_acc = nullptr;
  Adj adj() const { return Adj{adj_in, adj_ov}; }
};

namespace {

int lut3_rows(double d) {
  const double vol = kPi * d * d * d / 6.0, cap = kPi / (3.0 * std::sqrt(2.0));
  return (int)(cap / vol) + 2;  // every count from the last row on is held at the densest packing
}

// Per-count table of the 3-D step in FP64, in the oracle's operation order
// (the sphere volume fraction n pi d^3 / 6 held at pi / (3 sqrt 2), Eq. 9 at
// it, Eq. 20 at the voidage, the drag-law constants of Eqs. 19, 21, 22).
std::vector<double> build_lut3(const lbdps3_params &p) {
  const int rows = lut3_rows(p.d_p);
  std::vector<double> L((size_t)rows * L3_W, 0.0);
  const double d = p.d_p, vol = kPi * d * d * d / 6.0, cap = kPi / (3.0 * std::sqrt(2.0));
  const double mu = p.rho_g * ((p.tau - 0.5) / 3.0);
  for (int n = 0; n < rows; ++n) {
    double es = (double)n * vol;
    if (es > cap) es = cap;
    const double eg = 1.0 - es;
    const double gam = es * (p.tau - 0.5) / ((1.0 - es) + (p.tau - 0.5));
    const double om = eg > 0.74 ? omega_emms(eg) : p.omega_dense;
    double *r = &L[(size_t)n * L3_W];
    r[L3_ES] = es;
    r[L3_RELAX] = (1.0 - gam) / p.tau;
    r[L3_OMG] = om * gam;
    r[L3_EG] = eg;
    r[L3_DILUTE] = eg > 0.74 ? 1.0 : 0.0;
    r[L3_A] = 18.0 * (1.0 - eg) * om * mu / (d * d);
    r[L3_BRE] = eg * p.rho_g;
    r[L3_H] = 0.75 * (1.0 - eg) * eg * p.rho_g;
    r[L3_OM] = om;
    r[L3_D1] = 150.0 * (1.0 - eg) * (1.0 - eg) * mu / (eg * d * d);
    r[L3_D2] = 1.75 * (1.0 - eg) * p.rho_g;
  }
  return L;
}

size_t carve3(const lbdps3_params &p, long long nmax, char *base, lbdps3_ctx *x) {
  Carver cv{base};
  const int prec = p.precision;
  const size_t sS = prec == PREC_FP64 ? 8 : (prec == PREC_FP32 ? 4 : 2), sT = prec == PREC_FP64 ? 8 : 4;
  const size_t C = (size_t)p.nx * p.ny * p.nz, N = (size_t)std::max(nmax, 1ll);
  auto raw = [&](size_t bytes) { return cv.take<char>(bytes); };
  char *f0 = raw(Q3 * C * sS), *f1 = raw(Q3 * C * sS);
  char *fl[10];
  for (int i = 0; i < 9; ++i) fl[i] = raw(C * sT);
  fl[9] = raw(8 * C * sT);  // packed interpolation nodes
  int32_t *key[2], *pid[2];
  char *pos[2][3], *vel[2][3];
  for (int b = 0; b < 2; ++b) {
    key[b] = cv.take<int32_t>(N);
    pid[b] = cv.take<int32_t>(N);
    for (int a = 0; a < 3; ++a) pos[b][a] = raw(N * sT);
    for (int a = 0; a < 3; ++a) vel[b][a] = raw(N * sT);
  }
  int32_t *count = cv.take<int32_t>(C), *cs = cv.take<int32_t>(C + 1), *rank = cv.take<int32_t>(N);
  int32_t *slot = cv.take<int32_t>(N), *deg = cv.take<int32_t>(N), *done = cv.take<int32_t>(N);
  long long *adj_in = cv.take<long long>(N * ADJ_IN), *adj_ov = cv.take<long long>(N * (KMAX - ADJ_IN));
  int32_t *ticket = cv.take<int32_t>(4), *flags = cv.take<int32_t>(FLAG_COUNT);
  int32_t *chunk_busy = cv.take<int32_t>(N / RES_CHUNK + 1);
  const size_t tiles = (std::max(C, N) + SCAN_TILE - 1) / SCAN_TILE + 1;
  int32_t *spart = cv.take<int32_t>(tiles), *pcnt = cv.take<int32_t>(N + 1);
  const size_t nb = (size_t)nblocks((long long)std::max(C, N)) + 1;
  long long *pair_part = cv.take<long long>(nb), *coll_part = cv.take<long long>(nb);
  long long *collc_part = cv.take<long long>(nb);
  double *cpc = cv.take<double>(NB_CONS * 4), *cpp = cv.take<double>(NB_CONS * 3), *cout = cv.take<double>(8);
  int32_t *cflag = cv.take<int32_t>(4);
  const size_t nbN3 = (size_t)nblocks((long long)N);
  long long *roots = cv.take<long long>(nbN3 * BLOCK);
  int32_t *rcount = cv.take<int32_t>(nbN3), *need_sweep = cv.take<int32_t>(4);
  char *lut = raw((size_t)lut3_rows(p.d_p) * L3_W * sT);
  int32_t *dg_n = nullptr;
  char *dg_fd = nullptr, *dg_acc = nullptr;
  if (p.diagnostics) {
    dg_n = cv.take<int32_t>(C);
    dg_fd = raw(3 * N * sT);
    dg_acc = raw(3 * N * sT);
  }
  if (x) {
    x->f[0] = f0;
    x->f[1] = f1;
    for (int i = 0; i < 10; ++i) x->fld[i] = fl[i];
    for (int b = 0; b < 2; ++b) {
      x->key[b] = key[b];
      x->pid[b] = pid[b];
      for (int a = 0; a < 3; ++a) {
        x->pos[b][a] = pos[b][a];
        x->vel[b][a] = vel[b][a];
      }
    }
    x->count = count;
    x->cs = cs;
    x->rank = rank;
    x->slot = slot;
    x->deg = deg;
    x->done = done;
    x->adj_in = adj_in;
    x->adj_ov = adj_ov;
    x->ticket = ticket;
    x->flags = flags;
    x->chunk_busy = chunk_busy;
    x->spart = spart;
    x->pcnt = pcnt;
    x->pair_part = pair_part;
    x->coll_part = coll_part;
    x->collc_part = collc_part;
    x->cons_pc = cpc;
    x->cons_pp = cpp;
    x->cons_out = cout;
    x->cons_flag = cflag;
    x->roots = roots;
    x->rcount = rcount;
    x->need_sweep = need_sweep;
    x->lut = lut;
    x->dg_n = dg_n;
    x->dg_fd = dg_fd;
    x->dg_acc = dg_acc;
  }
  return cv.off + 256;
}

template <int P> struct Impl3 {
  using T = typename Prec<P>::T;
  using S = typename Prec<P>::S;
  static constexpr int kP = P;

  static Consts3<T> consts(const lbdps3_ctx *x) {
    Consts3<T> k{};
    k.nx = x->nx;
    k.ny = x->ny;
    k.nz = x->nz;
    k.C = x->C;
    k.npart = (int)x->n;
    k.nlut = x->nlut;
    k.tau = (T)x->dtau;
    k.d = (T)x->p.d_p;
    k.dd = (T)x->dd;
    k.mu = (T)x->dmu;
    k.vp = (T)x->dvp;
    k.m = (T)x->dm;
    k.msum = (T)(x->dm + x->dm);
    k.one_e = (T)x->done_e;
    k.fp = (T)x->dfp;
    for (int a = 0; a < 3; ++a) {
      k.geff[a] = (T)x->dgeff[a];
      k.halfG[a] = (T)x->dhalfG[a];
    }
    for (int i = 0; i < Q3; ++i) k.src[i] = (T)x->dsrc[i];
    k.flags = x->flags;
    k.spin_limit = 1u << 22;
    return k;
  }
  static Parts3<T> parts(const lbdps3_ctx *x, int b) {
    return Parts3<T>{x->key[b], x->pid[b], (T *)x->pos[b][0], (T *)x->pos[b][1], (T *)x->pos[b][2],
                     (T *)x->vel[b][0], (T *)x->vel[b][1], (T *)x->vel[b][2]};
  }
  static Fields3<T> fields(const lbdps3_ctx *x) {
    T *q[10];
    for (int i = 0; i < 10; ++i) q[i] = (T *)x->fld[i];
    return Fields3<T>{q[0], q[1], q[2], q[3], q[4], q[5], q[6], q[7], q[8], q[9]};
  }
  static void scan(lbdps3_ctx *x, int32_t *in, long long n, int32_t *out, int zero_in) {
    const int tiles = (int)((n + SCAN_TILE - 1) / SCAN_TILE) + (n == 0);
    hipLaunchKernelGGL(k_scan_reduce, dim3(tiles), dim3(BLOCK), 0, x->stream, in, n, x->spart);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(BLOCK), 0, x->stream, x->spart, tiles, out + n);
    hipLaunchKernelGGL(k_scan_apply, dim3(tiles), dim3(BLOCK), 0, x->stream, in, n, x->spart, out, zero_in);
  }
  // Cell starts of the records' current keys, then the records in cell order.
  static void sort(lbdps3_ctx *x, bool counted) {
    const int N = (int)x->n;
    if (!counted)
      hipLaunchKernelGGL(k3c_count<T>, dim3(nblocks(N)), dim3(BLOCK), 0, x->stream, parts(x, x->cp), N, x->count,
                         x->rank);
    scan(x, x->count, x->C, x->cs, 1);
    if (N > 0)
      hipLaunchKernelGGL(k3c_scatter<T>, dim3(nblocks(N)), dim3(BLOCK), 0, x->stream, parts(x, x->cp),
                         parts(x, 1 - x->cp), (const int32_t *)x->rank, (const int32_t *)x->cs, N, x->slot);
    x->cp = 1 - x->cp;
    x->bins_valid = true;
  }
  static void hard_spheres(lbdps3_ctx *x) {
    const int N = (int)x->n;
    if (N == 0) return;
    const Consts3<T> k = consts(x);
    hipLaunchKernelGGL(k3c_contacts<P>, dim3(nblocks(N)), dim3(BLOCK), 0, x->stream, parts(x, x->cp),
                       (const int32_t *)x->cs, k, x->adj(), x->deg, x->done, x->ticket, x->chunk_busy, x->pair_part,
                       x->need_sweep, x->roots, x->rcount);
    hipLaunchKernelGGL(k3c_clusters<P>, dim3(cluster_blocks(N, RC3_LISTS)), dim3(BLOCK), 0, x->stream,
                       parts(x, x->cp), x->adj(), (const int32_t *)x->deg, x->done, k, x->need_sweep, x->collc_part,
                       (const long long *)x->roots, (const int32_t *)x->rcount, nblocks(N));
    hipLaunchKernelGGL(k3c_resolve<P>, dim3(std::min(nblocks(N), 2048)), dim3(BLOCK), 0, x->stream, parts(x, x->cp),
                       (const int32_t *)x->slot, x->adj(), (const int32_t *)x->deg, x->done, x->ticket, k,
                       x->coll_part, x->chunk_busy, (const int32_t *)x->need_sweep);
  }
  static lbdps_status step(lbdps3_ctx *x, int nsteps) {
    const bool dg = x->p.diagnostics != 0;
    for (int it = 0; it < nsteps; ++it) {
      if (!x->bins_valid) sort(x, false);
      const Consts3<T> k = consts(x);
      hipLaunchKernelGGL(k3c_collide<P>, dim3(nblocks(x->C)), dim3(BLOCK), 0, x->stream, (const S *)x->f[x->cf],
                         (S *)x->f[1 - x->cf], fields(x), (const int32_t *)x->cs, parts(x, x->cp), (const T *)x->lut,
                         k, dg ? x->dg_n : nullptr);
      if (x->n > 0) {
        hipLaunchKernelGGL(k3c_gradp<P>, dim3(nblocks(x->C)), dim3(BLOCK), 0, x->stream, fields(x), k);
        // the moved records go to the other set, which then holds the current state
        hipLaunchKernelGGL(k3c_drag<P>, dim3(nblocks(x->n)), dim3(BLOCK), 0, x->stream, parts(x, x->cp),
                           parts(x, 1 - x->cp), fields(x), (const int32_t *)x->cs, k, x->count, x->rank,
                           dg ? (T *)x->dg_fd : nullptr, dg ? (T *)x->dg_acc : nullptr);
        x->cp = 1 - x->cp;
        sort(x, true);
        hard_spheres(x);
      }
      x->cf = 1 - x->cf;
      x->step += 1;
    }
    return launch_status("lbdps3_step");
  }
  static lbdps_status set_state(lbdps3_ctx *x, const double *d_f, const double *d_pos, const double *d_vel,
                                long long n) {
    const long long e = (long long)Q3 * x->C;
    hipLaunchKernelGGL(k3_set_f<P>, dim3((unsigned)((e + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, x->stream, d_f,
                       (S *)x->f[x->cf], x->C);
    x->n = n;
    const Consts3<T> k = consts(x);
    if (n > 0)
      hipLaunchKernelGGL(k3c_set_parts<P>, dim3(nblocks(n)), dim3(BLOCK), 0, x->stream, d_pos, d_vel, (int)n,
                         parts(x, x->cp), k);
    x->bins_valid = false;
    x->step = 0;
    if (x->p.diagnostics)
      hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(x->C)), dim3(BLOCK), 0, x->stream, x->dg_n, (long long)x->C, 0);
    return launch_status("lbdps3_set_state");
  }
  static void get_state(lbdps3_ctx *x, double *d_f, double *d_pos, double *d_vel) {
    const long long e = (long long)Q3 * x->C;
    if (d_f)
      hipLaunchKernelGGL(k3_get_f<P>, dim3((unsigned)((e + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, x->stream,
                         (const S *)x->f[x->cf], d_f, x->C);
    if (x->n > 0 && (d_pos || d_vel)) {
      if (!x->bins_valid) sort(x, false);
      hipLaunchKernelGGL(k3c_get_parts<P>, dim3(nblocks(x->n)), dim3(BLOCK), 0, x->stream, parts(x, x->cp),
                         (const int32_t *)x->slot, (int)x->n, consts(x), d_pos, d_vel);
    }
  }
  static void get_field(lbdps3_ctx *x, const void *a, const void *b, const void *c, double *out, double add,
                        long long n) {
    hipLaunchKernelGGL(k3_get_field<T>, dim3(nblocks(n)), dim3(BLOCK), 0, x->stream, (const T *)a, (const T *)b,
                       (const T *)c, n, out, add);
  }
};

template <class F> lbdps_status dispatch3(lbdps3_ctx *x, F &&fn) {
  switch (x->prec) {
    case PREC_FP64: return fn(Impl3<PREC_FP64>{});
    case PREC_FP32: return fn(Impl3<PREC_FP32>{});
    case PREC_FP16DEV: return fn(Impl3<PREC_FP16DEV>{});
    case PREC_BF16DEV: return fn(Impl3<PREC_BF16DEV>{});
  }
  return fail(LBDPS_E_INVALID, "unknown precision");
}

lbdps_status sync3(lbdps3_ctx *x, const char *what) {
  lbdps_status st = check_hip(hipStreamSynchronize(x->stream), what);
  if (st != LBDPS_OK) return st;
  int32_t fl[FLAG_COUNT];
  st = check_hip(hipMemcpy(fl, x->flags, sizeof(fl), hipMemcpyDeviceToHost), what);
  if (st != LBDPS_OK) return st;
  bool any = false;
  for (int i = 0; i < FLAG_COUNT; ++i) any |= fl[i] != 0;
  if (!any) return LBDPS_OK;
  const int32_t zero[FLAG_COUNT] = {0};
  check_hip(hipMemcpy(x->flags, zero, sizeof(zero), hipMemcpyHostToDevice), what);
  if (fl[FLAG_DOMAIN]) return fail(LBDPS_E_INVALID, std::string(what) + ": a particle was placed outside the box");
  if (fl[FLAG_CAPACITY])
    return fail(LBDPS_E_CAPACITY, std::string(what) + ": a particle had more than LBDPS_MAX_CONTACTS contacts");
  if (fl[FLAG_STALL]) return fail(LBDPS_E_STALL, std::string(what) + ": collision resolution exceeded its wait bound");
  return fail(LBDPS_E_DEVICE, std::string(what) + ": unknown device flag");
}

}  // namespace

extern "C" {

lbdps_status lbdps3_validate_params(const lbdps3_params *p, int64_t max_particles) {
  if (!p) return fail(LBDPS_E_INVALID, "params is NULL");
  if (p->nx < 3 || p->ny < 3 || p->nz < 3) return fail(LBDPS_E_SHAPE, "nx, ny and nz must be >= 3");
  if ((long long)p->nx * p->ny * p->nz >= (1ll << 28)) return fail(LBDPS_E_SHAPE, "nx * ny * nz must be < 2^28");
  if (!(is_fin(p->tau) && p->tau > 0.5)) return fail(LBDPS_E_INVALID, "tau must be > 0.5");
  if (!(is_fin(p->rho_g) && p->rho_g > 0)) return fail(LBDPS_E_INVALID, "rho_g must be > 0");
  if (!(is_fin(p->rho_s) && p->rho_s > 0)) return fail(LBDPS_E_INVALID, "rho_s must be > 0");
  if (!(is_fin(p->d_p) && p->d_p >= 0.1 && p->d_p < 1.0)) return fail(LBDPS_E_INVALID, "d_p must be in [0.1, 1)");
  if (!(p->e_pp >= 0 && p->e_pp <= 1)) return fail(LBDPS_E_INVALID, "e_pp must be in [0, 1]");
  for (int a = 0; a < 3; ++a)
    if (!is_fin(p->g[a]) || !is_fin(p->body_force[a])) return fail(LBDPS_E_INVALID, "g and body_force must be finite");
  if (!is_fin(p->omega_dense)) return fail(LBDPS_E_INVALID, "omega_dense must be finite");
  if (p->pressure_force_sign < -1 || p->pressure_force_sign > 1)
    return fail(LBDPS_E_INVALID, "pressure_force_sign must be -1, 0 or 1");
  if (p->precision < 0 || p->precision > 3) return fail(LBDPS_E_INVALID, "precision must be 0..3");
  if (p->diagnostics < 0 || p->diagnostics > 1) return fail(LBDPS_E_INVALID, "diagnostics must be 0 or 1");
  if (max_particles < 0 || max_particles >= (1ll << 28)) return fail(LBDPS_E_SHAPE, "max_particles must be in [0, 2^28)");
  return LBDPS_OK;
}

lbdps_status lbdps3_workspace_bytes(const lbdps3_params *p, int64_t max_particles, size_t *bytes) {
  lbdps_status st = lbdps3_validate_params(p, max_particles);
  if (st != LBDPS_OK) return st;
  if (!bytes) return fail(LBDPS_E_INVALID, "bytes is NULL");
  *bytes = carve3(*p, max_particles, nullptr, nullptr);
  return LBDPS_OK;
}

lbdps_status lbdps3_create(const lbdps3_params *p, int64_t max_particles, void *d_workspace, size_t bytes,
                           void *stream, lbdps3_ctx **out) {
  if (!out) return fail(LBDPS_E_INVALID, "out is NULL");
  *out = nullptr;
  lbdps_status st = lbdps3_validate_params(p, max_particles);
  if (st != LBDPS_OK) return st;
  const size_t need = carve3(*p, max_particles, nullptr, nullptr);
  if (!d_workspace) return fail(LBDPS_E_INVALID, "workspace is NULL");
  if (bytes < need) return fail(LBDPS_E_SHAPE, "workspace too small: need " + std::to_string(need) + " bytes");
  if (((uintptr_t)d_workspace & 255) != 0) return fail(LBDPS_E_INVALID, "workspace must be 256-byte aligned");
  lbdps3_ctx *x = new (std::nothrow) lbdps3_ctx();
  if (!x) return fail(LBDPS_E_DEVICE, "host allocation failed");
  x->p = *p;
  x->prec = p->precision;
  x->nx = p->nx;
  x->ny = p->ny;
  x->nz = p->nz;
  x->C = p->nx * p->ny * p->nz;
  x->nmax = max_particles;
  x->nlut = lut3_rows(p->d_p);
  x->stream = (hipStream_t)stream;
  x->dtau = p->tau;
  x->dd = p->d_p * p->d_p;
  x->dmu = p->rho_g * ((p->tau - 0.5) / 3.0);
  x->dvp = kPi * p->d_p * p->d_p * p->d_p / 6.0;
  x->dm = p->rho_s * x->dvp;
  x->done_e = 1.0 + p->e_pp;
  x->dfp = (double)p->pressure_force_sign * x->dvp;
  for (int a = 0; a < 3; ++a) {
    x->dgeff[a] = (1.0 - p->rho_g / p->rho_s) * p->g[a];
    x->dhalfG[a] = 0.5 * p->body_force[a];
  }
  for (int i = 0; i < Q3; ++i)
    x->dsrc[i] = 3.0 * w3<double>(i) *
                 (c3(i, 0) * p->body_force[0] + c3(i, 1) * p->body_force[1] + c3(i, 2) * p->body_force[2]);
  carve3(*p, max_particles, (char *)d_workspace, x);
  std::vector<double> lut = build_lut3(*p);
  if (x->prec == PREC_FP64) {
    st = check_hip(hipMemcpy(x->lut, lut.data(), lut.size() * 8, hipMemcpyHostToDevice), "lbdps3_create");
  } else {
    std::vector<float> lf(lut.begin(), lut.end());
    st = check_hip(hipMemcpy(x->lut, lf.data(), lf.size() * 4, hipMemcpyHostToDevice), "lbdps3_create");
  }
  if (st != LBDPS_OK) {
    delete x;
    return st;
  }
  hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(x->C)), dim3(BLOCK), 0, x->stream, x->count, (long long)x->C, 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(BLOCK), 0, x->stream, x->flags, (long long)FLAG_COUNT, 0);
  hipLaunchKernelGGL(k_fill_i32, dim3(nblocks(x->nmax / RES_CHUNK + 1)), dim3(BLOCK), 0, x->stream, x->chunk_busy,
                     (long long)(x->nmax / RES_CHUNK + 1), 0);
  st = dispatch3(x, [&](auto impl) { return decltype(impl)::set_state(x, nullptr, nullptr, nullptr, 0); });
  if (st == LBDPS_OK) st = check_hip(hipStreamSynchronize(x->stream), "lbdps3_create");
  if (st != LBDPS_OK) {
    delete x;
    return st;
  }
  *out = x;
  return LBDPS_OK;
}

lbdps_status lbdps3_set_state(lbdps3_ctx *x, const double *d_f, const double *d_pos, const double *d_vel,
                              int64_t n) {
  if (!x) return fail(LBDPS_E_INVALID, "ctx is NULL");
  if (n < 0 || n > x->nmax) return fail(LBDPS_E_SHAPE, "n must be in [0, max_particles]");
  if (n > 0 && (!d_pos || !d_vel)) return fail(LBDPS_E_INVALID, "positions and velocities are required when n > 0");
  return dispatch3(x, [&](auto impl) { return decltype(impl)::set_state(x, d_f, d_pos, d_vel, n); });
}

lbdps_status lbdps3_step(lbdps3_ctx *x, int32_t nsteps) {
  if (!x) return fail(LBDPS_E_INVALID, "ctx is NULL");
  if (nsteps < 0) return fail(LBDPS_E_INVALID, "nsteps must be >= 0");
  return dispatch3(x, [&](auto impl) { return decltype(impl)::step(x, nsteps); });
}

lbdps_status lbdps3_get_state(lbdps3_ctx *x, double *d_f, double *d_pos, double *d_vel) {
  if (!x) return fail(LBDPS_E_INVALID, "ctx is NULL");
  lbdps_status st = dispatch3(x, [&](auto impl) {
    decltype(impl)::get_state(x, d_f, d_pos, d_vel);
    return launch_status("lbdps3_get_state");
  });
  if (st != LBDPS_OK) return st;
  return sync3(x, "lbdps3_get_state");
}

lbdps_status lbdps3_get_fields(lbdps3_ctx *x, double *d_rho, double *d_ugas, double *d_fpg, double *d_beta,
                               int32_t *d_ncell) {
  if (!x) return fail(LBDPS_E_INVALID, "ctx is NULL");
  if (d_ncell && !x->p.diagnostics) return fail(LBDPS_E_INVALID, "n_tot needs diagnostics on");
  lbdps_status st = dispatch3(x, [&](auto impl) {
    using I = decltype(impl);
    const double add = x->prec == PREC_FP64 ? 0.0 : 1.0;  // the deviation modes keep rho - 1
    if (d_rho) I::get_field(x, x->fld[0], nullptr, nullptr, d_rho, add, x->C);
    if (d_ugas) I::get_field(x, x->fld[1], x->fld[2], x->fld[3], d_ugas, 0.0, x->C);
    if (d_beta) I::get_field(x, x->fld[4], nullptr, nullptr, d_beta, 0.0, x->C);
    if (d_fpg) I::get_field(x, x->fld[6], x->fld[7], x->fld[8], d_fpg, 0.0, x->C);
    if (d_ncell)
      (void)check_hip(hipMemcpyAsync(d_ncell, x->dg_n, (size_t)x->C * 4, hipMemcpyDeviceToDevice, x->stream),
                      "lbdps3_get_fields");
    return launch_status("lbdps3_get_fields");
  });
  if (st != LBDPS_OK) return st;
  return sync3(x, "lbdps3_get_fields");
}

lbdps_status lbdps3_get_drag(lbdps3_ctx *x, double *d_fd, double *d_acc) {
  if (!x) return fail(LBDPS_E_INVALID, "ctx is NULL");
  if (!x->p.diagnostics) return fail(LBDPS_E_INVALID, "the drag is recorded with diagnostics on");
  if (x->n > 0) {
    lbdps_status st = dispatch3(x, [&](auto impl) {
      using I = decltype(impl);
      if (d_fd) I::get_field(x, x->dg_fd, nullptr, nullptr, d_fd, 0.0, 3 * x->n);
      if (d_acc) I::get_field(x, x->dg_acc, nullptr, nullptr, d_acc, 0.0, 3 * x->n);
      return launch_status("lbdps3_get_drag");
    });
    if (st != LBDPS_OK) return st;
  }
  return sync3(x, "lbdps3_get_drag");
}

lbdps_status lbdps3_get_pairs(lbdps3_ctx *x, int32_t *d_pairs, int64_t cap, int64_t *n_out) {
  if (!x || !n_out) return fail(LBDPS_E_INVALID, "ctx or n_out is NULL");
  if (cap < 0 || (cap > 0 && !d_pairs)) return fail(LBDPS_E_INVALID, "bad pair buffer");
  const int N = (int)x->n;
  *n_out = 0;
  if (N == 0) return sync3(x, "lbdps3_get_pairs");
  hipLaunchKernelGGL(k_pairs_count, dim3(nblocks(N)), dim3(BLOCK), 0, x->stream, x->slot, x->adj(), x->deg, N,
                     x->rank);
  dispatch3(x, [&](auto impl) {
    decltype(impl)::scan(x, x->rank, N, x->pcnt, 0);
    return LBDPS_OK;
  });
  hipLaunchKernelGGL(k_pairs_write, dim3(nblocks(N)), dim3(BLOCK), 0, x->stream, x->slot, x->adj(), x->deg, N,
                     x->pcnt, d_pairs, (long long)cap);
  lbdps_status st = launch_status("lbdps3_get_pairs");
  if (st != LBDPS_OK) return st;
  int32_t total = 0;
  st = check_hip(hipMemcpyAsync(&total, x->pcnt + N, 4, hipMemcpyDeviceToHost, x->stream), "lbdps3_get_pairs");
  if (st != LBDPS_OK) return st;
  st = sync3(x, "lbdps3_get_pairs");
  *n_out = total;
  return st;
}

lbdps_status lbdps3_counters(lbdps3_ctx *x, int64_t h_out[2]) {
  if (!x || !h_out) return fail(LBDPS_E_INVALID, "ctx or out is NULL");
  lbdps_status st = sync3(x, "lbdps3_counters");
  if (st != LBDPS_OK) return st;
  h_out[0] = h_out[1] = 0;
  if (x->n == 0) return LBDPS_OK;
  const int nb = nblocks(x->n), nr = std::min(nblocks(x->n), 2048);
  std::vector<long long> buf((size_t)nb);
  st = check_hip(hipMemcpy(buf.data(), x->pair_part, (size_t)nb * 8, hipMemcpyDeviceToHost), "lbdps3_counters");
  if (st != LBDPS_OK) return st;
  for (int b = 0; b < nb; ++b) h_out[0] += buf[b];
  st = check_hip(hipMemcpy(buf.data(), x->coll_part, (size_t)nr * 8, hipMemcpyDeviceToHost), "lbdps3_counters");
  if (st != LBDPS_OK) return st;
  for (int b = 0; b < nr; ++b) h_out[1] += buf[b];
  const int ncl = cluster_blocks(x->n, RC3_LISTS);
  st = check_hip(hipMemcpy(buf.data(), x->collc_part, (size_t)ncl * 8, hipMemcpyDeviceToHost), "lbdps3_counters");
  if (st != LBDPS_OK) return st;
  for (int b = 0; b < ncl; ++b) h_out[1] += buf[b];
  return LBDPS_OK;
}

lbdps_status lbdps3_conservation(lbdps3_ctx *x, double h_out[8]) {
  if (!x || !h_out) return fail(LBDPS_E_INVALID, "ctx or out is NULL");
  lbdps_status st = dispatch3(x, [&](auto impl) {
    using I = decltype(impl);
    using T = typename I::T;
    using S = typename I::S;
    const double mass = x->p.rho_s * kPi * x->p.d_p * x->p.d_p * x->p.d_p / 6.0;
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(BLOCK), 0, x->stream, x->cons_flag, 1ll, 0);
    hipLaunchKernelGGL(k3_cons_cells<decltype(impl)::kP>, dim3(NB_CONS), dim3(BLOCK), 0, x->stream,
                       (const S *)x->f[x->cf], (long long)x->C, x->cons_pc, x->cons_flag);
    hipLaunchKernelGGL(k3_cons_parts<T>, dim3(NB_CONS), dim3(BLOCK), 0, x->stream, I::parts(x, x->cp), (int)x->n,
                       mass, x->cons_pp, x->cons_flag);
    hipLaunchKernelGGL(k3_cons_final, dim3(1), dim3(BLOCK), 0, x->stream, (const double *)x->cons_pc, NB_CONS,
                       (const double *)x->cons_pp, NB_CONS, (const int32_t *)x->cons_flag, x->cons_out);
    return launch_status("lbdps3_conservation");
  });
  if (st != LBDPS_OK) return st;
  st = check_hip(hipMemcpyAsync(h_out, x->cons_out, 8 * sizeof(double), hipMemcpyDeviceToHost, x->stream),
                 "lbdps3_conservation");
  if (st != LBDPS_OK) return st;
  st = sync3(x, "lbdps3_conservation");
  if (st != LBDPS_OK) return st;
  if (h_out[7] != 0.0) return fail(LBDPS_E_NONFINITE, "non-finite value in populations or velocities");
  return LBDPS_OK;
}

lbdps_status lbdps3_destroy(lbdps3_ctx *x) {
  if (!x) return fail(LBDPS_E_INVALID, "ctx is NULL");
  (void)hipStreamSynchronize(x->stream);
  delete x;
  return LBDPS_OK;
}

}  // extern "C"
