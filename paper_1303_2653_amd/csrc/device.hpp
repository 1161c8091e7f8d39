// Device-side building blocks for gfx950: precision traits, D2Q9 constants,
// kernel argument structs.  Wave64 throughout.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbdps {

constexpr int Q = 9;
constexpr int KMAX = 32;      // contacts stored per particle
constexpr int BLOCK = 256;    // threads per workgroup (4 waves)
constexpr int LUT_W = 12;     // columns of the per-count table

// Eight wavefronts per SIMD (at most 64 VGPRs) for the drag and contact
// kernels: they are bound by memory round trips, and one more resident
// wavefront per SIMD hides more of them than the registers it costs (5 % and
// 3 % on a 16 M-particle bed).  The cluster kernel spills at 64 VGPRs and
// runs slower, so it keeps its own register count.
#define LBDPS_WAVES8 __attribute__((amdgpu_waves_per_eu(8, 8)))
// Six wavefronts per SIMD (at most 80 VGPRs) for the drag kernel's flat form,
// which holds up to three particles per thread: 9 % faster than its natural
// 86 VGPRs and five wavefronts on a 16 M-particle bed, with no spills.
#define LBDPS_WAVES6 __attribute__((amdgpu_waves_per_eu(6, 6)))

// The launch's workgroups are dealt to the chip's eight XCDs in turn (dispatch
// index i runs on XCD i mod 8), and each XCD has an L2 of its own.
// xcd_block<R> maps the dispatch index to a tile index so that each XCD takes
// runs of R consecutive tiles: neighbouring tiles, which read the same cache
// lines of neighbouring cells and particles, then share an L2.  R = 0 gives
// each XCD one contiguous run of the whole launch; R < 0 keeps the dispatch
// order.  Short runs keep the XCDs' loads even where the work is spread
// unevenly over the tiles.  A bijection of [0, gdim) for any gdim: with R > 0
// the last, partial group of 8 R tiles keeps the dispatch order.
constexpr int NXCD = 8;
template <int R> __host__ __device__ constexpr int xcd_block(int bid, int gdim) {
  if constexpr (R < 0) {
    return bid;
  } else if constexpr (R == 0) {
    return (bid % NXCD) * (gdim / NXCD) + (bid % NXCD < gdim % NXCD ? bid % NXCD : gdim % NXCD) + bid / NXCD;
  } else {
    constexpr int G = NXCD * R;
    return bid >= gdim - gdim % G ? bid : bid - bid % G + (bid % NXCD) * R + (bid % G) / NXCD;
  }
}
// Run lengths per kernel.  The kernels that gather from neighbouring rows
// (drag, contacts, cluster resolution) take runs of 8 tiles: measured against
// the dispatch order, their time drops 4-10 % on a 16.8 M-cell bed and on a
// batch of uneven beds, where one run per XCD left some XCDs idle.  The
// streaming kernels keep the dispatch order.
constexpr int XCD_RUN_COLLIDE = -1, XCD_RUN_DRAG = 8, XCD_RUN_SCAN = -1, XCD_RUN_SCATTER = -1,
              XCD_RUN_CONTACTS = 8, XCD_RUN_CLUSTERS = 8, XCD_RUN_RESOLVE = -1;

enum { BC_PERIODIC = 0, BC_WALL = 1, BC_INLET = 2, BC_OUTLET = 3 };
enum { PREC_FP64 = 0, PREC_FP32 = 1, PREC_FP16DEV = 2, PREC_BF16DEV = 3 };
// Error flag slots (int32 each).
enum { FLAG_DOMAIN = 0, FLAG_CAPACITY = 1, FLAG_STALL = 2, FLAG_NONFINITE = 3, FLAG_COUNT = 8 };
// Columns of the per-count table (built on the host in FP64).
enum {
  L_ES3 = 0,  // 3-D solid fraction eps_s,3d (Eq. 11)
  L_UDIV,     // divisor turning the superficial into the actual gas velocity
  L_OMG,      // omega * gamma (Eqs. 9, 20, 23)
  L_RELAX,    // (1 - gamma) / tau (Eq. 23)
  L_A,        // dilute low-Re drag prefactor 18 (1-eg) omega mu / d^2
  L_BRE,      // eg * rho_g  (Re_p = eg rho_g |u-v| d / mu, Eq. 22)
  L_H,        // 0.75 (1-eg) eg rho_g  (dilute, Re_p >= 1000)
  L_OM,       // omega (Eq. 20)
  L_D1,       // Ergun viscous term 150 (1-eg)^2 mu / (eg d^2)
  L_D2,       // Ergun inertial prefactor 1.75 (1-eg) rho_g
  L_DILUTE,   // 1 if eg > 0.74
  L_ES2       // 2-D solid fraction eps_s,2d (Eq. 10), for gamma at tau_t (Eq. 9)
};

// D2Q9, numbering 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1).
__host__ __device__ constexpr int cx_of(int i) {
  return i == 1 || i == 5 || i == 8 ? 1 : (i == 3 || i == 6 || i == 7 ? -1 : 0);
}
__host__ __device__ constexpr int cy_of(int i) {
  return i == 2 || i == 5 || i == 6 ? 1 : (i == 4 || i == 7 || i == 8 ? -1 : 0);
}
__host__ __device__ constexpr int opp9(int i) {
  return i == 0 ? 0 : i == 1 ? 3 : i == 2 ? 4 : i == 3 ? 1 : i == 4 ? 2 : i == 5 ? 7 : i == 6 ? 8 : i == 7 ? 5 : 6;
}
template <class T>
__host__ __device__ constexpr T wgt(int i) {
  return i == 0 ? T(4.0 / 9.0) : (i <= 4 ? T(1.0 / 9.0) : T(1.0 / 36.0));
}

// bf16 <-> fp32 with round-to-nearest-even.
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Precision modes: T = arithmetic type, S = population storage type.  In the
// deviation modes a population is stored as f_i - w_i.  In FP64 particle
// positions are global coordinates; otherwise a cell index plus an offset in
// [0, 1) (so FP32 keeps its resolution on tall lattices).
template <int P> struct Prec;
template <> struct Prec<PREC_FP64> {
  using T = double;
  using S = double;
  static constexpr bool global_pos = true;
};
template <> struct Prec<PREC_FP32> {
  using T = float;
  using S = float;
  static constexpr bool global_pos = false;
};
template <> struct Prec<PREC_FP16DEV> {
  using T = float;
  using S = _Float16;
  static constexpr bool global_pos = false;
};
template <> struct Prec<PREC_BF16DEV> {
  using T = float;
  using S = uint16_t;
  static constexpr bool global_pos = false;
};

// Stored population value: f_i itself in FP64; in the reduced precisions the
// deviation g_i = f_i - w_i from the lattice weight, so that moments of
// populations close to the weights keep their digits in single precision.
template <int P> constexpr bool kDev = P != PREC_FP64;

template <int P>
__device__ __forceinline__ typename Prec<P>::T load_v(const typename Prec<P>::S *f, size_t idx) {
  if constexpr (P == PREC_FP64 || P == PREC_FP32) return f[idx];
  else if constexpr (P == PREC_FP16DEV) return (float)f[idx];
  else return bf16_to_f32(f[idx]);
}

template <int P>
__device__ __forceinline__ void store_v(typename Prec<P>::S *f, size_t idx, typename Prec<P>::T v) {
  if constexpr (P == PREC_FP64 || P == PREC_FP32) f[idx] = v;
  else if constexpr (P == PREC_FP16DEV) f[idx] = (_Float16)v;  // round to nearest even
  else f[idx] = f32_to_bf16(v);
}

// Population i as FP64 f_i (canonical value).
template <int P> __device__ __forceinline__ double to_f64(const typename Prec<P>::S *f, size_t idx, int i) {
  if constexpr (kDev<P>) return wgt<double>(i) + (double)load_v<P>(f, idx);
  else return (double)f[idx];
}

template <int P> __device__ __forceinline__ void from_f64(typename Prec<P>::S *f, size_t idx, int i, double v) {
  using T = typename Prec<P>::T;
  if constexpr (kDev<P>) store_v<P>(f, idx, (T)(v - wgt<double>(i)));
  else f[idx] = v;
}

// Scalar constants of a context, in the arithmetic type.
template <class T> struct Consts {
  int nx, ny, C, nlut;
  unsigned long long nx_m;  // key / nx = (key * nx_m) >> nx_s for 0 <= key < 2^31
  int nx_s;
  int per_x, per_y, bc_ylo, bc_yhi;  // per_y: the particles' periodicity along y
  int gas_per_y;                     // the lattice's periodicity along y
  int drag_abs;
  int drag_reg;  // Eq. 28 with the equal split where a cell's pre-drags cancel
  int npart;
  T tau, d, mu, vp, m, msum, one_e, e_pw, r;
  int les;  // Smagorinsky sub-grid model on (Eqs. 12-15)
  T cs18;   // 18 C_s^2 of Eq. 15
  T geff[2], fp, halfG[2], src[Q];
  T h;          // particle sub-step length, 1 / n_sub
  T *acx, *acy; // accelerations held over the lattice step by particle index (n_sub > 1), else null
  unsigned spin_limit;
  int32_t *flags;                // the context's latched device error flags
  unsigned long long *cross;     // running net count of particles across y = ny upward (outlet flux)
};

// Cell row of a key: key / nx by one multiplication and shift.  With
// s = 31 + ceil(log2 nx) and m = ceil(2^s / nx), m nx = 2^s + e with 0 <= e < nx,
// so key m / 2^s exceeds key / nx by less than 1 / nx and the floors agree for
// every key < 2^31 (Granlund & Montgomery, division by invariant integers).
template <class T> __device__ __forceinline__ int cell_row(const Consts<T> &k, int key) {
  return (int)(((unsigned long long)(unsigned)key * k.nx_m) >> k.nx_s);
}
template <class T> __device__ __forceinline__ void cell_xy(const Consts<T> &k, int key, int &cx, int &cy) {
  cy = cell_row(k, key);
  cx = key - cy * k.nx;
}

// Division, square root and power in the arithmetic type.  FP64 keeps the
// correctly rounded operations exactly as written (the oracle's results bit for
// bit); the modes with FP32 arithmetic use the hardware reciprocal, square root,
// log2 and exp2 instructions (about 1 ulp each).
template <int P, class T> __device__ __forceinline__ T dv(T a, T b) {
  if constexpr (P == PREC_FP64) return a / b;
  else return a * __builtin_amdgcn_rcpf(b);
}
template <int P, class T> __device__ __forceinline__ T sq(T a) {
  if constexpr (P == PREC_FP64) return sqrt(a);
  else return __builtin_amdgcn_sqrtf(a);
}
template <int P, class T> __device__ __forceinline__ T pw(T a, T e) {
  if constexpr (P == PREC_FP64) return pow(a, e);
  else return __builtin_amdgcn_exp2f(e * __builtin_amdgcn_logf(a));
}

// Element i of an array whose base address is uniform across the wavefront,
// addressed by a 32-bit byte offset: the load then takes the base from scalar
// registers and one 32-bit vector offset, with no 64-bit address arithmetic
// per lane.  Needs 0 <= i and i * sizeof(T) < 2^32 (the library bounds the
// particle count and the lattice size at creation).
template <class T> __device__ __forceinline__ T ldu(const T *base, int i) {
  return *(const T *)((const char *)base + (unsigned)i * (unsigned)sizeof(T));
}

// Particle storage (structure of arrays, one "slot" per particle).
template <class T> struct Parts {
  int32_t *key;  // cell index y * nx + x
  int32_t *pid;  // particle index (orders the collisions)
  T *px, *py;    // global position (FP64) or offset in the cell (reduced precisions)
  T *vx, *vy;
};

// Node fields written by the collision, read by the particle stage.
template <class T> struct Fields {
  T *rho, *ugx, *ugy, *beta, *fpgx, *fpgy, *es;  // es: 3-D solid fraction of the node (Eq. 11)
};

}  // namespace lbdps
