/*
 * lbdps oracle: a plain, slow FP64 CPU implementation of one time step of the
 * lattice-Boltzmann-based discrete particle simulation of Wang, Zhang, Wang,
 * Ge & Li, "Lattice Boltzmann based discrete simulation for gas-solid
 * fluidization" (Chem. Eng. Sci.).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  The GPU library never
 * links, includes or calls it, and the two share no code.
 *
 * Build: gcc -std=c99 -O2 -ffp-contract=off -fPIC -shared -o liboracle.so lbdps_oracle.c -lm
 * (contraction off, so every product and sum below is one IEEE operation).
 * The same command with -fopenmp gives liboracle_omp.so, whose per-cell loops
 * run on all host cores with bit-identical results (ORC_CELLS_PARALLEL).
 *
 * Units: lattice units, h = dt = 1, so c = h/dt = 1 (note after Eq. 14),
 * c_s^2 = 1/3 (Sec. 2.1, text after Eq. 4) and every h^2/dt factor is 1 (Eq. 25).
 *
 * Interpretations of points the paper leaves open are numbered R1..R44 in the
 * design notes; the comment at each use says which one applies.
 *
 * Parity status: every function is pinned by a closed form, an invariant,
 * printed values or brute force in tests/test_oracle_*.py.  The drag
 * coefficient beta is pinned branch by branch against the textbook laws it is
 * built from (Ergun's pressure drop, the Wen & Yu force per sphere with its
 * voidage function in place of omega, Schiller & Naumann's single-sphere
 * drag); the EMMS factor omega itself only by the extreme values printed with
 * Eq. 20.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* R49: the cancellation bound of the regularised Eq. 28 (drag_ratio_mode 2) */
#define ORC_CANCEL_MAX 100.0

#define ORC_PERIODIC 0
#define ORC_WALL 1
#define ORC_INLET 2  /* equilibrium incoming populations (R21) */
#define ORC_OUTLET 3 /* zero-gradient (R22) */

static const double PI = 3.14159265358979323846;

/* The per-cell loops marked with this are independent from cell to cell.
 * Built with -fopenmp (liboracle_omp.so, the all-cores CPU baseline) they are
 * spread over the host's cores; each cell's arithmetic is unchanged, so the
 * results are bit-identical to the plain build, which ignores the pragma.
 * Particle loops and every sum over particles stay sequential. */
#define ORC_CELLS_PARALLEL _Pragma("omp parallel for schedule(static)")

/* Threads the per-cell loops use: 1 in the plain build. */
int32_t orc_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

#define ORC_OK 0
#define ORC_E_DOMAIN (-1)
#define ORC_E_CAPACITY (-6)

typedef struct {
  int32_t nx, ny;
  int32_t bc[4]; /* faces x-, x+, y-, y+ */
  double tau;
  double rho_g, rho_s, d;
  double e_pp, e_pw;
  double g[2];   /* gravity acting on particles, before the (1 - rho_g/rho_s) factor */
  double G[2];   /* body force on the gas per cell (R29) */
  int32_t drag_ratio_mode; /* 0 signed (R15), 1 literal absolute values, 2 signed with
                              the equal split where the pre-drags cancel (R49) */
  int32_t u_gas_porosity;  /* 0 divide by eps_2d, 1 by eps_g (3-D), 2 none (R6) */
  int32_t omega_mode;      /* 0 EMMS Eq. 20, 1 omega == 1 everywhere (Eq. 6) */
  int32_t pressure_sign;   /* -1 physical (R17), 0 off, +1 as printed in Eq. 16 */
  double omega_dense;      /* omega for eps_g <= 0.74 (R9) */
  double cs_smag;          /* Smagorinsky constant, 0 = plain BGK (Eqs. 12-15) */
  int32_t n_sub;           /* particle sub-steps per lattice step, 0 or 1 = one (R41) */
  int32_t particles_periodic_y; /* 1: particles leaving through a non-periodic y face re-enter at the
                                   other one (the circulating loop of Sec. 3.2, R44); the gas keeps
                                   its faces */
} orc_params;

typedef struct {
  int32_t *ncell; /* [C]    particles per cell (Eq. 8's n_tot) */
  double *vs;     /* [C][2] cell-average solid velocity (Eq. 8) */
  double *rho;    /* [C]    density (Eq. 5) */
  double *ugas;   /* [C][2] actual gas velocity (Eq. 24 and the note after it) */
  double *fpg;    /* [C][2] force of the particles on the gas (Eq. 25) */
  double *beta;   /* [C]    EMMS drag coefficient at the node (Eq. 19) */
  double *fd;     /* [N][2] corrected drag on each particle (Eq. 28) */
  double *fpre;   /* [N][2] pre-estimated drag (Eq. 26) */
  double *upart;  /* [N][2] gas velocity interpolated at the particle */
  double *acc;    /* [N][2] acceleration of Eq. 16 (held over the sub-steps, R41) */
  int32_t *pairs; /* [cap][2] contact pairs after the move, lexicographic */
  int64_t pair_cap;
  int64_t npairs;      /* out */
  int64_t ncollisions; /* out: pairs that were approaching and collided */
  int64_t nwall;       /* out: particle-wall collisions */
  int64_t nzero_den;   /* out: cell components where Eq. 28's denominator was 0 */
  int64_t ncross;      /* out: net particles across the outlet plane y = ny, upward (R47) */
} orc_out;

/* ---- D2Q9 lattice (Sec. 2.1, text after Eq. 4), diagonals as (+-1, +-1) (R1) ---- */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double W[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

void orc_lattice(int32_t *c, double *w, int32_t *opp) {
  for (int i = 0; i < 9; ++i) {
    c[2 * i] = CX[i];
    c[2 * i + 1] = CY[i];
    w[i] = W[i];
    opp[i] = OPP[i];
  }
}

/* Eq. 4 with c_s^2 = 1/3: 1/c_s^2 = 3, 1/(2 c_s^4) = 4.5, 1/(2 c_s^2) = 1.5. */
double orc_feq(int i, double rho, double ux, double uy) {
  double cu = CX[i] * ux + CY[i] * uy;
  double uu = ux * ux + uy * uy;
  return W[i] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
}

/* Eq. 9. */
double orc_gamma(double eps_s, double tau) {
  return eps_s * (tau - 0.5) / ((1.0 - eps_s) + (tau - 0.5));
}

/* Eq. 20, defined for eps_g > 0.74; the breakpoints 0.82 and 0.97 belong to the
 * lower branch as printed (R32). */
double orc_omega_emms(double eg) {
  if (eg <= 0.82) {
    double t = eg - 0.7463;
    return 0.0214 / (4.0 * t * t + 0.0044) - 0.5760;
  }
  if (eg <= 0.97) {
    double t = eg - 0.7789;
    return 0.0038 / (4.0 * t * t + 0.0040) - 0.0101;
  }
  return 32.8295 * eg - 31.8295;
}

/* Eq. 21, literal (used by the tests only; the step uses the rewrite of R12). */
double orc_cd0(double re) {
  if (re < 1000.0) return 24.0 / re * (1.0 + 0.15 * pow(re, 0.687));
  return 0.44;
}

/* Eq. 11's coefficient sqrt(2)/sqrt(pi sqrt(3)). */
static double eps3_coeff(void) { return sqrt(2.0) / sqrt(PI * sqrt(3.0)); }

/* Gas viscosity: tau = 3 nu + 1/2 (Eq. 3), mu_g = rho_g nu with the constant
 * parameter rho_g (R12). */
static double mu_gas(const orc_params *p) { return p->rho_g * ((p->tau - 0.5) / 3.0); }

/*
 * Solid statistics of a cell holding n particle centres:
 *   out[0] eps_s,2d = n pi r^2 / h^2 (Eq. 10), clamped at the densest disc
 *          packing pi/(2 sqrt 3) (R7)
 *   out[1] eps_2d   = 1 - eps_s,2d
 *   out[2] eps_s,3d = coeff * eps_s,2d^(3/2) (Eq. 11)
 *   out[3] eps_g    = 1 - eps_s,3d, the voidage of the drag laws (R10)
 *   out[4] gamma(eps_s,2d, tau) (Eq. 9)
 *   out[5] omega: Eq. 20 at eps_g when eps_g > 0.74, else omega_dense (R9);
 *          1 when omega_mode == 1
 */
void orc_cell_props(const orc_params *p, int64_t n, double *out) {
  double disc = PI * p->d * p->d / 4.0;
  double es2 = (double)n * disc;
  double cap = PI / (2.0 * sqrt(3.0));
  if (es2 > cap) es2 = cap;
  double es3 = eps3_coeff() * pow(es2, 1.5);
  double eg = 1.0 - es3;
  double om;
  if (p->omega_mode == 1)
    om = 1.0;
  else if (eg > 0.74)
    om = orc_omega_emms(eg);
  else
    om = p->omega_dense;
  out[0] = es2;
  out[1] = 1.0 - es2;
  out[2] = es3;
  out[3] = eg;
  out[4] = orc_gamma(es2, p->tau);
  out[5] = om;
}

/*
 * EMMS drag coefficient (Eq. 19) with C_d0 from Eq. 21 and Re_p from Eq. 22,
 * at voidage eg, correction om and slip speed |u - v|.  For Re_p < 1000 the
 * dilute branch is written with Re_p cancelled, 18 (1-eg) om mu / d^2
 * (1 + 0.15 Re^0.687), which equals 3/4 (1-eg) eg rho |u-v| / d * C_d0 * om
 * exactly and is finite at Re_p = 0 (R12).
 */
double orc_beta(const orc_params *p, double eg, double om, double slip) {
  double mu = mu_gas(p);
  double d = p->d;
  if (eg > 0.74) {
    double re = eg * p->rho_g * slip * d / mu;
    if (re < 1000.0) return 18.0 * (1.0 - eg) * om * mu / (d * d) * (1.0 + 0.15 * pow(re, 0.687));
    return 0.75 * (1.0 - eg) * eg * p->rho_g * slip * 0.44 * om / d;
  }
  return 150.0 * (1.0 - eg) * (1.0 - eg) * mu / (eg * d * d) + 1.75 * (1.0 - eg) * p->rho_g * slip / d;
}

/*
 * Relaxation time of the BGK part with the Smagorinsky sub-grid model
 * (Eqs. 12-15).  The momentum flux of the non-equilibrium populations,
 * Q_ij = sum_k c_ki c_kj (f_k - f_k^eq) (Eq. 13), with f^eq at the raw moment
 * velocity (R5), has the norm Q = sqrt(2 Q_ij Q_ij).  Eq. 13 gives the strain
 * rate S = Q / (2 rho c_s^2 tau_t), Eq. 12 the eddy viscosity
 * nu_e = C_s^2 S (dx = 1) and Eq. 14 tau_t = 3 (nu + nu_e) + 1/2 = tau + 3 nu_e;
 * together tau_t^2 - tau tau_t - 9 C_s^2 Q / (2 rho) = 0, whose positive root is
 * Eq. 15 with Q / rho in place of the printed Q (R40; rho is close to 1).
 * With C_s = 0 this is tau itself (LES off, R30).
 */
double orc_tau_les(const orc_params *p, const double *f, const double *feq, double rho) {
  if (p->cs_smag == 0.0) return p->tau;
  double qxx = 0.0, qyy = 0.0, qxy = 0.0;
  for (int i = 0; i < 9; ++i) {
    double ne = f[i] - feq[i];
    qxx += CX[i] * CX[i] * ne;
    qyy += CY[i] * CY[i] * ne;
    qxy += CX[i] * CY[i] * ne;
  }
  double q = sqrt(2.0 * (qxx * qxx + qyy * qyy + 2.0 * (qxy * qxy)));
  double cs18 = 18.0 * p->cs_smag * p->cs_smag;
  return 0.5 * (p->tau + sqrt(p->tau * p->tau + cs18 * q / rho));
}

/*
 * Collision at one node, Eq. 23 with tau_t from orc_tau_les (R4: the BGK part
 * relaxes with 1/tau_t and gamma(eps_s, tau_t), the solid term keeps
 * gamma(eps_s, tau)), the solid term of Eq. 7 and the gas body-force source of
 * R29.
 *   f[9]      pre-collision populations
 *   n, vs[2]  particles in the cell and their mean velocity (Eq. 8, R8)
 *   fstar[9]  post-collision populations
 *   o[0] rho (Eq. 5)
 *   o[1..2] actual gas velocity u_gas = u_sup / eps (Eq. 24 and note, R6)
 *   o[3..4] F_p->g (Eq. 25)
 *   o[5] beta at the node (Eq. 19) with slip |u_gas - vs|
 *   o[6..7] superficial velocity u_sup (Eq. 24)
 * Equilibria use the plain moment velocity u = sum(c f)/rho (R5).
 */
void orc_collide_node(const orc_params *p, const double *f, int64_t n, const double *vs, double *fstar,
                      double *o) {
  double pr[6];
  orc_cell_props(p, n, pr);
  double gam = pr[4], om = pr[5];
  double rho = 0.0, jx = 0.0, jy = 0.0;
  for (int i = 0; i < 9; ++i) rho += f[i];
  for (int i = 0; i < 9; ++i) jx += CX[i] * f[i];
  for (int i = 0; i < 9; ++i) jy += CY[i] * f[i];
  double ux = jx / rho, uy = jy / rho;
  double fu[9], fv[9], oms[9];
  for (int i = 0; i < 9; ++i) {
    fu[i] = orc_feq(i, rho, ux, uy);
    fv[i] = orc_feq(i, rho, vs[0], vs[1]);
  }
  /* Eq. 7 */
  for (int i = 0; i < 9; ++i) oms[i] = f[OPP[i]] - f[i] + fv[i] - fu[OPP[i]];
  double omg = om * gam;
  double relax = (1.0 - gam) / p->tau;
  if (p->cs_smag != 0.0) {  /* Eqs. 12-15 (R40) */
    double tt = orc_tau_les(p, f, fu, rho);
    relax = (1.0 - orc_gamma(pr[0], tt)) / tt;
  }
  for (int i = 0; i < 9; ++i) {
    double src = 3.0 * W[i] * (CX[i] * p->G[0] + CY[i] * p->G[1]);
    fstar[i] = f[i] - relax * (f[i] - fu[i]) + omg * oms[i] + src;
  }
  /* Eq. 25 */
  double sx = 0.0, sy = 0.0;
  for (int i = 0; i < 9; ++i) sx += CX[i] * oms[i];
  for (int i = 0; i < 9; ++i) sy += CY[i] * oms[i];
  double fx = omg * sx, fy = omg * sy;
  /* Eq. 24: rho u_sup = sum c (f + omg Om/2) (+ G/2 for the body force, R29) */
  double usx = (jx + 0.5 * fx + 0.5 * p->G[0]) / rho;
  double usy = (jy + 0.5 * fy + 0.5 * p->G[1]) / rho;
  double ugx = usx, ugy = usy;
  if (p->u_gas_porosity == 0) {
    ugx = usx / pr[1];
    ugy = usy / pr[1];
  } else if (p->u_gas_porosity == 1) {
    ugx = usx / pr[3];
    ugy = usy / pr[3];
  }
  double dx = ugx - vs[0], dy = ugy - vs[1];
  double slip = sqrt(dx * dx + dy * dy);
  o[0] = rho;
  o[1] = ugx;
  o[2] = ugy;
  o[3] = fx;
  o[4] = fy;
  o[5] = orc_beta(p, pr[3], om, slip);
  o[6] = usx;
  o[7] = usy;
}

static int is_periodic_x(const orc_params *p) { return p->bc[0] == ORC_PERIODIC; }
static int is_periodic_y(const orc_params *p) { return p->bc[2] == ORC_PERIODIC; }
/* Periodicity of the particles along y: that of the gas, or the circulating
 * loop (R44). */
static int particles_periodic_y(const orc_params *p) { return is_periodic_y(p) || p->particles_periodic_y; }

/* Node index along x for interpolation and gradients: wrap on periodic axes,
 * clamp into [0, nx-1] otherwise (R11, R17). */
static int node_x(const orc_params *p, int i) {
  if (is_periodic_x(p)) return ((i % p->nx) + p->nx) % p->nx;
  return i < 0 ? 0 : (i >= p->nx ? p->nx - 1 : i);
}
static int node_y(const orc_params *p, int j) {
  if (is_periodic_y(p)) return ((j % p->ny) + p->ny) % p->ny;
  return j < 0 ? 0 : (j >= p->ny ? p->ny - 1 : j);
}

/*
 * Streaming, pull form: f_i(x, t+1) = f*_i(x - c_i), with boundary rules:
 *   x faces: periodic, or halfway bounce-back (walls at x = 0 and x = nx), and an
 *     x wall takes precedence over a y face at corners (R20);
 *   y faces: periodic, bounce-back, equilibrium inlet f^eq(1, (0, u_in(x))) (R21),
 *     or zero-gradient outlet taking f*_i from the boundary row (R22).
 * fstar and fnew are [9][ny][nx].
 */
void orc_stream(const orc_params *p, const double *inlet_uy, const double *fstar, double *fnew) {
  const int nx = p->nx, ny = p->ny;
  const int64_t C = (int64_t)nx * ny;
  ORC_CELLS_PARALLEL
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      int64_t c = (int64_t)y * nx + x;
      for (int i = 0; i < 9; ++i) {
        int sx = x - CX[i], sy = y - CY[i];
        double val;
        if (sx < 0 || sx >= nx) {
          if (!is_periodic_x(p)) {
            fnew[i * C + c] = fstar[OPP[i] * C + c];
            continue;
          }
          sx = (sx + nx) % nx;
        }
        if (sy < 0 || sy >= ny) {
          int face = sy < 0 ? p->bc[2] : p->bc[3];
          if (face == ORC_PERIODIC) {
            sy = (sy + ny) % ny;
          } else if (face == ORC_WALL) {
            fnew[i * C + c] = fstar[OPP[i] * C + c];
            continue;
          } else if (face == ORC_INLET) {
            double uin = inlet_uy ? inlet_uy[x] : 0.0;
            fnew[i * C + c] = orc_feq(i, 1.0, 0.0, uin);
            continue;
          } else { /* outlet: zero gradient, source row is the boundary row */
            sy = sy < 0 ? 0 : ny - 1;
          }
        }
        val = fstar[i * C + (int64_t)sy * nx + sx];
        fnew[i * C + c] = val;
      }
    }
}

/* Bilinear stencil around a particle (R11): nodes sit at cell centres (i+1/2,
 * j+1/2); s = P - (1/2, 1/2), i0 = floor(s_x), t_x = s_x - i0.  idx = the four
 * node indices (i0,j0), (i0+1,j0), (i0,j0+1), (i0+1,j0+1); wt = their weights. */
void orc_stencil(const orc_params *p, double px, double py, int64_t *idx, double *wt) {
  double sx = px - 0.5, sy = py - 0.5;
  double fx = floor(sx), fy = floor(sy);
  double tx = sx - fx, ty = sy - fy;
  int i0 = (int)fx, j0 = (int)fy;
  int ia = node_x(p, i0), ib = node_x(p, i0 + 1);
  int ja = node_y(p, j0), jb = node_y(p, j0 + 1);
  idx[0] = (int64_t)ja * p->nx + ia;
  idx[1] = (int64_t)ja * p->nx + ib;
  idx[2] = (int64_t)jb * p->nx + ia;
  idx[3] = (int64_t)jb * p->nx + ib;
  wt[0] = (1.0 - tx) * (1.0 - ty);
  wt[1] = tx * (1.0 - ty);
  wt[2] = (1.0 - tx) * ty;
  wt[3] = tx * ty;
}

/* Bilinear interpolation of a node field q[C] at (px, py) (Sec. 2.3, after Eq. 26). */
double orc_interp(const orc_params *p, const double *q, double px, double py) {
  int64_t idx[4];
  double wt[4];
  orc_stencil(p, px, py, idx, wt);
  return wt[0] * q[idx[0]] + wt[1] * q[idx[1]] + wt[2] * q[idx[2]] + wt[3] * q[idx[3]];
}

/* Node pressure gradient by central differences of p = rho c_s^2, with the
 * ghost beyond a non-periodic face equal to the boundary value (R17).
 * pres[C] in, grad[C][2] out. */
void orc_grad_p(const orc_params *p, const double *pres, double *grad) {
  const int nx = p->nx, ny = p->ny;
  ORC_CELLS_PARALLEL
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      int64_t c = (int64_t)y * nx + x;
      double pe = pres[(int64_t)y * nx + node_x(p, x + 1)];
      double pw = pres[(int64_t)y * nx + node_x(p, x - 1)];
      double pn = pres[(int64_t)node_y(p, y + 1) * nx + x];
      double ps = pres[(int64_t)node_y(p, y - 1) * nx + x];
      grad[2 * c] = (pe - pw) * 0.5;
      grad[2 * c + 1] = (pn - ps) * 0.5;
    }
}

/* Particle constants: V_p = pi d^3 / 6, m = rho_s V_p (R19), effective gravity
 * (1 - rho_g/rho_s) g (Sec. 3, first paragraph). */
static double vol_p(const orc_params *p) { return PI * p->d * p->d * p->d / 6.0; }
static double mass_p(const orc_params *p) { return p->rho_s * vol_p(p); }

/* Periodic wrap of one coordinate (R26). */
static double wrap_coord(double x, double L) {
  if (x >= L) {
    x -= L;
  } else if (x < 0.0) {
    x += L;
    if (x >= L) x = 0.0;
  }
  return x;
}

/* Mirror a coordinate that crossed a wall plane at 0 or L back inside (R23). */
static double mirror_coord(double x, double L) {
  if (x < 0.0) x = -x;
  if (x >= L) x = 2.0 * L - x;
  if (x >= L) x = nextafter(L, 0.0);
  return x;
}

/*
 * Acceleration of Eq. 16 for every particle:
 *   a = g_eff + (F_d + s V_p grad p_k) / m,
 * with s = pressure_sign (R17).  fd[N][2] and gpk[N][2] are the drag and the
 * interpolated pressure gradient; acc[N][2] receives a.
 */
static void accelerations(const orc_params *p, int64_t np, const double *fd, const double *gpk, double *acc) {
  double vp = vol_p(p), m = mass_p(p);
  double fp = (double)p->pressure_sign * vp;
  double gex = (1.0 - p->rho_g / p->rho_s) * p->g[0];
  double gey = (1.0 - p->rho_g / p->rho_s) * p->g[1];
  for (int64_t k = 0; k < np; ++k) {
    acc[2 * k] = gex + (fd[2 * k] + fp * gpk[2 * k]) / m;
    acc[2 * k + 1] = gey + (fd[2 * k + 1] + fp * gpk[2 * k + 1]) / m;
  }
}

/*
 * One symplectic Euler step of length h (R18): v <- v + a h, P <- P + v h, then
 * periodic wrap (R26) or wall mirror (R23).  Returns the net number of
 * particles that crossed the plane y = ny upward in the move (R47): with
 * particles periodic in y, +1 for a move that ends at y >= ny (wrapped to the
 * bottom), -1 for one that ends below 0; 0 when y has walls.
 */
static int64_t advance(const orc_params *p, int64_t np, double *pos, double *vel, const double *acc, double h) {
  int64_t cross = 0;
  for (int64_t k = 0; k < np; ++k) {
    vel[2 * k] = vel[2 * k] + acc[2 * k] * h;
    vel[2 * k + 1] = vel[2 * k + 1] + acc[2 * k + 1] * h;
    double x = pos[2 * k] + vel[2 * k] * h;
    double y = pos[2 * k + 1] + vel[2 * k + 1] * h;
    x = is_periodic_x(p) ? wrap_coord(x, p->nx) : mirror_coord(x, p->nx);
    if (particles_periodic_y(p)) {
      if (y >= (double)p->ny)
        ++cross;
      else if (y < 0.0)
        --cross;
      y = wrap_coord(y, p->ny);
    } else {
      y = mirror_coord(y, p->ny);
    }
    pos[2 * k] = x;
    pos[2 * k + 1] = y;
  }
  return cross;
}

/*
 * Eq. 16 integrated with symplectic Euler over one whole step, dt_p = 1 (R18):
 *   v <- v + g_eff + (F_d + s V_p grad p_k) / m,   P <- P + v.
 */
void orc_integrate(const orc_params *p, int64_t np, double *pos, double *vel, const double *fd,
                   const double *gpk) {
  double *acc = (double *)malloc((size_t)(np > 0 ? np : 1) * 2 * sizeof(double));
  accelerations(p, np, fd, gpk, acc);
  advance(p, np, pos, vel, acc, 1.0);
  free(acc);
}

/* Outlet solids mass flux of Sec. 3.2 from the net number of particles that
 * crossed the outlet plane y = ny upward over `steps` steps (R47): the mass
 * m = rho_s pi d^3 / 6 they carry per unit width of the outlet (unit depth,
 * h = 1) per unit time (dt = 1). */
double orc_solids_flux(const orc_params *p, int64_t net, int64_t steps) {
  return mass_p(p) * (double)net / ((double)p->nx * (double)steps);
}

/* Minimum-image separation P_i - P_j along each axis (R25). */
static void separation(const orc_params *p, const double *a, const double *b, double *dx, double *dy) {
  double x = a[0] - b[0], y = a[1] - b[1];
  if (is_periodic_x(p)) {
    if (x > 0.5 * p->nx)
      x -= p->nx;
    else if (x < -0.5 * p->nx)
      x += p->nx;
  }
  if (particles_periodic_y(p)) {
    if (y > 0.5 * p->ny)
      y -= p->ny;
    else if (y < -0.5 * p->ny)
      y += p->ny;
  }
  *dx = x;
  *dy = y;
}

/* Contact predicate (Sec. 2.2): centres no farther apart than d, ties count (R25). */
static int in_contact(const orc_params *p, const double *a, const double *b) {
  double dx, dy;
  separation(p, a, b, &dx, &dy);
  return dx * dx + dy * dy <= p->d * p->d;
}

static int cmp_pair(const void *a, const void *b) {
  const int32_t *x = (const int32_t *)a, *y = (const int32_t *)b;
  if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
  if (x[1] != y[1]) return x[1] < y[1] ? -1 : 1;
  return 0;
}

/* All pairs i < j in contact, by testing every pair; lexicographic order. */
int orc_contacts_brute(const orc_params *p, int64_t np, const double *pos, int32_t *pairs, int64_t cap,
                       int64_t *npairs) {
  int64_t m = 0;
  for (int64_t i = 0; i < np; ++i)
    for (int64_t j = i + 1; j < np; ++j)
      if (in_contact(p, pos + 2 * i, pos + 2 * j)) {
        if (m >= cap) {
          *npairs = m;
          return ORC_E_CAPACITY;
        }
        pairs[2 * m] = (int32_t)i;
        pairs[2 * m + 1] = (int32_t)j;
        ++m;
      }
  *npairs = m;
  return ORC_OK;
}

/* Cell-list bucketing: members of cell c are list[start[c] .. start[c+1]) in
 * ascending particle index.  cell[k] is the cell of particle k. */
static void bucket(int64_t C, int64_t np, const int32_t *cell, int64_t *start, int64_t *list) {
  for (int64_t c = 0; c <= C; ++c) start[c] = 0;
  for (int64_t k = 0; k < np; ++k) start[cell[k] + 1]++;
  for (int64_t c = 0; c < C; ++c) start[c + 1] += start[c];
  int64_t *fill = (int64_t *)malloc((size_t)(C + 1) * sizeof(int64_t));
  memcpy(fill, start, (size_t)(C + 1) * sizeof(int64_t));
  for (int64_t k = 0; k < np; ++k) list[fill[cell[k]]++] = k;
  free(fill);
}

/* The same set as orc_contacts_brute, found through 1x1-cell bins (valid for
 * d < 1: a contact partner lies in one of the 3x3 cells around a particle). */
int orc_contacts_cells(const orc_params *p, int64_t np, const double *pos, int32_t *pairs, int64_t cap,
                       int64_t *npairs) {
  const int nx = p->nx, ny = p->ny;
  const int64_t C = (int64_t)nx * ny;
  int32_t *cell = (int32_t *)malloc((size_t)(np > 0 ? np : 1) * sizeof(int32_t));
  int64_t *start = (int64_t *)malloc((size_t)(C + 1) * sizeof(int64_t));
  int64_t *list = (int64_t *)malloc((size_t)(np > 0 ? np : 1) * sizeof(int64_t));
  for (int64_t k = 0; k < np; ++k) {
    int cx = (int)floor(pos[2 * k]), cy = (int)floor(pos[2 * k + 1]);
    cell[k] = cy * nx + cx;
  }
  bucket(C, np, cell, start, list);
  int64_t m = 0;
  int rc = ORC_OK;
  for (int64_t i = 0; i < np && rc == ORC_OK; ++i) {
    int cx = cell[i] % nx, cy = cell[i] / nx;
    for (int oy = -1; oy <= 1 && rc == ORC_OK; ++oy)
      for (int ox = -1; ox <= 1 && rc == ORC_OK; ++ox) {
        int x = cx + ox, y = cy + oy;
        if (x < 0 || x >= nx) {
          if (!is_periodic_x(p)) continue;
          x = (x + nx) % nx;
        }
        if (y < 0 || y >= ny) {
          if (!particles_periodic_y(p)) continue;
          y = (y + ny) % ny;
        }
        int64_t c = (int64_t)y * nx + x;
        for (int64_t s = start[c]; s < start[c + 1]; ++s) {
          int64_t j = list[s];
          if (j <= i) continue;
          if (in_contact(p, pos + 2 * i, pos + 2 * j)) {
            if (m >= cap) {
              rc = ORC_E_CAPACITY;
              break;
            }
            pairs[2 * m] = (int32_t)i;
            pairs[2 * m + 1] = (int32_t)j;
            ++m;
          }
        }
      }
  }
  qsort(pairs, (size_t)m, 2 * sizeof(int32_t), cmp_pair);
  *npairs = m;
  free(cell);
  free(start);
  free(list);
  return rc;
}

/*
 * Contact predicate in single precision on a cell + offset position state (R25,
 * R27): cell[k][2] integer cell, off[k][2] float offset in [0, 1).  The cell
 * difference takes the periodic minimum image as an integer; then
 * dx = (float)dcx + (off_i - off_j) and dx*dx + dy*dy <= d*d, each operation
 * rounded to float.  brute != 0 tests all pairs; otherwise 3x3 cell bins.
 */
int orc_contacts_f32(int32_t nx, int32_t ny, int32_t per_x, int32_t per_y, float d, int64_t np,
                     const int32_t *cell, const float *off, int32_t brute, int32_t *pairs, int64_t cap,
                     int64_t *npairs) {
  const int64_t C = (int64_t)nx * ny;
  float dd = d * d;
  int64_t m = 0;
  int rc = ORC_OK;
  int32_t *key = (int32_t *)malloc((size_t)(np > 0 ? np : 1) * sizeof(int32_t));
  int64_t *start = (int64_t *)malloc((size_t)(C + 1) * sizeof(int64_t));
  int64_t *list = (int64_t *)malloc((size_t)(np > 0 ? np : 1) * sizeof(int64_t));
  for (int64_t k = 0; k < np; ++k) key[k] = cell[2 * k + 1] * nx + cell[2 * k];
  bucket(C, np, key, start, list);
  for (int64_t i = 0; i < np && rc == ORC_OK; ++i) {
    int64_t jlo = i + 1, jhi = np;
    int cells = brute ? 1 : 9;
    for (int q = 0; q < cells && rc == ORC_OK; ++q) {
      const int64_t *cand;
      int64_t ncand;
      if (brute) {
        cand = NULL;
        ncand = jhi - jlo;
      } else {
        int x = cell[2 * i] + (q % 3) - 1, y = cell[2 * i + 1] + (q / 3) - 1;
        if (x < 0 || x >= nx) {
          if (!per_x) continue;
          x = (x + nx) % nx;
        }
        if (y < 0 || y >= ny) {
          if (!per_y) continue;
          y = (y + ny) % ny;
        }
        int64_t c = (int64_t)y * nx + x;
        cand = list + start[c];
        ncand = start[c + 1] - start[c];
      }
      for (int64_t s = 0; s < ncand; ++s) {
        int64_t j = brute ? jlo + s : cand[s];
        if (j <= i) continue;
        int dcx = cell[2 * i] - cell[2 * j], dcy = cell[2 * i + 1] - cell[2 * j + 1];
        if (per_x) {
          if (dcx > nx / 2)
            dcx -= nx;
          else if (dcx < -(nx / 2))
            dcx += nx;
        }
        if (per_y) {
          if (dcy > ny / 2)
            dcy -= ny;
          else if (dcy < -(ny / 2))
            dcy += ny;
        }
        float ox = off[2 * i] - off[2 * j];
        float oy = off[2 * i + 1] - off[2 * j + 1];
        float dx = (float)dcx + ox;
        float dy = (float)dcy + oy;
        float r2 = dx * dx + dy * dy;
        if (r2 <= dd) {
          if (m >= cap) {
            rc = ORC_E_CAPACITY;
            break;
          }
          pairs[2 * m] = (int32_t)i;
          pairs[2 * m + 1] = (int32_t)j;
          ++m;
        }
      }
    }
  }
  qsort(pairs, (size_t)m, 2 * sizeof(int32_t), cmp_pair);
  *npairs = m;
  free(key);
  free(start);
  free(list);
  return rc;
}

/*
 * Hard-sphere collisions (Eqs. 17-18) over the contact pairs in the given
 * (lexicographic) order, each with the current velocities (R24).  A pair
 * collides only if (P_1 - P_2).(v_1 - v_2) < 0 (Sec. 2.2).  All particles share
 * one mass here, but the formula keeps m_1 and m_2 as printed.
 */
void orc_resolve(const orc_params *p, int64_t np, const double *pos, double *vel, const int32_t *pairs,
                 int64_t npairs, int64_t *ncoll) {
  (void)np;
  double m1 = mass_p(p), m2 = mass_p(p);
  int64_t nc = 0;
  for (int64_t q = 0; q < npairs; ++q) {
    int64_t i = pairs[2 * q], j = pairs[2 * q + 1];
    double dx, dy;
    separation(p, pos + 2 * i, pos + 2 * j, &dx, &dy);
    double dvx = vel[2 * i] - vel[2 * j], dvy = vel[2 * i + 1] - vel[2 * j + 1];
    double dot = dvx * dx + dvy * dy;
    if (!(dot < 0.0)) continue;
    double r2 = dx * dx + dy * dy;
    double q0 = (1.0 + p->e_pp) * dot / r2;
    double ci = q0 * m2 / (m1 + m2);
    double cj = q0 * m1 / (m1 + m2);
    vel[2 * i] = vel[2 * i] - ci * dx;
    vel[2 * i + 1] = vel[2 * i + 1] - ci * dy;
    vel[2 * j] = vel[2 * j] + cj * dx;
    vel[2 * j + 1] = vel[2 * j + 1] + cj * dy;
    ++nc;
  }
  if (ncoll) *ncoll = nc;
}

/*
 * Particle-wall collisions (Sec. 2.2, walls as infinitely heavy particles, and
 * the boundary rule of the procedure's step 1): on every non-periodic axis, a
 * particle within r of a wall and moving into it has its normal velocity
 * replaced by -e_w times itself (R23).  Faces in the order x-, x+, y-, y+.
 */
void orc_walls(const orc_params *p, int64_t np, const double *pos, double *vel, int64_t *nwall) {
  double r = 0.5 * p->d;
  int64_t nw = 0;
  for (int64_t k = 0; k < np; ++k) {
    double x = pos[2 * k], y = pos[2 * k + 1];
    if (!is_periodic_x(p)) {
      if (x <= r && vel[2 * k] < 0.0) {
        vel[2 * k] = -p->e_pw * vel[2 * k];
        ++nw;
      }
      if ((double)p->nx - x <= r && vel[2 * k] > 0.0) {
        vel[2 * k] = -p->e_pw * vel[2 * k];
        ++nw;
      }
    }
    if (!particles_periodic_y(p)) {
      if (y <= r && vel[2 * k + 1] < 0.0) {
        vel[2 * k + 1] = -p->e_pw * vel[2 * k + 1];
        ++nw;
      }
      if ((double)p->ny - y <= r && vel[2 * k + 1] > 0.0) {
        vel[2 * k + 1] = -p->e_pw * vel[2 * k + 1];
        ++nw;
      }
    }
  }
  if (nwall) *nwall = nw;
}

/*
 * The hard-sphere stage (Sec. 2.2) in single precision on a cell + offset
 * state (R25, R27, R46): the contact pairs of orc_contacts_f32 (cell bins),
 * then the binary collisions of Eqs. 17-18 over the pairs in lexicographic
 * order with the current velocities (R24), then the particle-wall collisions
 * (R23), every operation rounded to float in the order written:
 *   dx  = (float)dcx + (off_i - off_j), dcx the minimum-image cell difference
 *   dot = (v_ix - v_jx) dx + (v_iy - v_jy) dy;  the pair collides iff dot < 0
 *   q   = ((1 + e) dot) / (dx dx + dy dy)
 *   c   = (q m) / (m + m)       (m_j / (m_i + m_j) with one mass m)
 *   v_i <- v_i - c (dx, dy),  v_j <- v_j + c (dx, dy)
 * and, per particle in index order, on each non-periodic axis: in the first
 * cell with offset <= r, or in the last with 1 - offset <= r (r = d/2), and
 * moving into that wall, v_n <- -e_w v_n (face x- before x+).  1 + e, e_w,
 * r, d and m = rho_s pi d^3 / 6 are formed in FP64 and rounded to float once.
 * cell[N][2], off[N][2] (float, [0, 1)), vel[N][2] float in and out, index
 * order.  pairs[cap][2] receives the contact pairs; the counts go to
 * npairs, ncoll (pairs that collided) and nwall.
 */
int orc_collide_f32(int32_t nx, int32_t ny, int32_t per_x, int32_t per_y, double d, double rho_s, double e_pp,
                    double e_pw, int64_t np, const int32_t *cell, const float *off, float *vel, int32_t *pairs,
                    int64_t cap, int64_t *npairs, int64_t *ncoll, int64_t *nwall) {
  const float one_e = (float)(1.0 + e_pp), ew = (float)e_pw, r = (float)(0.5 * d);
  const float m = (float)(rho_s * (PI * d * d * d / 6.0));
  int rc = orc_contacts_f32(nx, ny, per_x, per_y, (float)d, np, cell, off, 0, pairs, cap, npairs);
  *ncoll = 0;
  *nwall = 0;
  if (rc != ORC_OK) return rc;
  for (int64_t q = 0; q < *npairs; ++q) {
    int64_t i = pairs[2 * q], j = pairs[2 * q + 1];
    int dcx = cell[2 * i] - cell[2 * j], dcy = cell[2 * i + 1] - cell[2 * j + 1];
    if (per_x) {
      if (dcx > nx / 2)
        dcx -= nx;
      else if (dcx < -(nx / 2))
        dcx += nx;
    }
    if (per_y) {
      if (dcy > ny / 2)
        dcy -= ny;
      else if (dcy < -(ny / 2))
        dcy += ny;
    }
    float ox = off[2 * i] - off[2 * j], oy = off[2 * i + 1] - off[2 * j + 1];
    float dx = (float)dcx + ox, dy = (float)dcy + oy;
    float dvx = vel[2 * i] - vel[2 * j], dvy = vel[2 * i + 1] - vel[2 * j + 1];
    float dot = dvx * dx + dvy * dy;
    if (!(dot < 0.0f)) continue;
    float r2 = dx * dx + dy * dy;
    float q0 = (one_e * dot) / r2;
    float c = (q0 * m) / (m + m);
    vel[2 * i] = vel[2 * i] - c * dx;
    vel[2 * i + 1] = vel[2 * i + 1] - c * dy;
    vel[2 * j] = vel[2 * j] + c * dx;
    vel[2 * j + 1] = vel[2 * j + 1] + c * dy;
    ++*ncoll;
  }
  for (int64_t k = 0; k < np; ++k) {
    float *v = vel + 2 * k;
    for (int a = 0; a < 2; ++a) {
      if (a == 0 ? per_x : per_y) continue;
      int c = cell[2 * k + a], n = a == 0 ? nx : ny;
      float o = off[2 * k + a];
      if (c == 0 && o <= r && v[a] < 0.0f) {
        v[a] = -ew * v[a];
        ++*nwall;
      }
      if (c == n - 1 && 1.0f - o <= r && v[a] > 0.0f) {
        v[a] = -ew * v[a];
        ++*nwall;
      }
    }
  }
  return ORC_OK;
}

/*
 * One coupled time step, the procedure of Sec. 2.4 (steps 2 to 6):
 *   2) per-cell particle count, mean solid velocity and porosities (Eqs. 8, 10, 11)
 *   3) collision (Eq. 23) with moments, F_p->g and beta (Eqs. 19-25), then streaming
 *   4) interpolation, pre-estimated drag (Eq. 26), per-cell sums (Eq. 27) and the
 *      corrected drag (Eq. 28)
 *   5) integration of Eq. 16
 *   6) contact detection at the new positions and binary collisions (Eqs. 17-18),
 *      then particle-wall collisions
 * With n_sub > 1 sub-steps (R41), 5) and 6) run n_sub times with h = 1 / n_sub
 * under the accelerations of step 4, held over the whole lattice step; the
 * pair list and the counters then describe the last sub-step.
 * f[9][ny][nx] (pre-collision, advanced in place), pos[N][2], vel[N][2] (id
 * order, advanced in place).  Per-cell sums run in ascending particle index (R28).
 */
int orc_step(const orc_params *p, const double *inlet_uy, double *f, int64_t np, double *pos, double *vel,
             orc_out *out) {
  const int nx = p->nx, ny = p->ny;
  const int64_t C = (int64_t)nx * ny;
  const size_t NP = (size_t)(np > 0 ? np : 1);
  int rc = ORC_OK;

  /* ---- 2) deposition ---- */
  int32_t *cell = (int32_t *)malloc(NP * sizeof(int32_t));
  int32_t *ncell = (int32_t *)calloc((size_t)C, sizeof(int32_t));
  double *sv = (double *)calloc((size_t)(2 * C), sizeof(double));
  for (int64_t k = 0; k < np; ++k) {
    double fx = floor(pos[2 * k]), fy = floor(pos[2 * k + 1]);
    if (!(fx >= 0.0 && fx < nx && fy >= 0.0 && fy < ny)) {
      rc = ORC_E_DOMAIN;
      break;
    }
    int32_t c = (int32_t)fy * nx + (int32_t)fx;
    cell[k] = c;
    ncell[c] += 1;
    sv[2 * c] += vel[2 * k];
    sv[2 * c + 1] += vel[2 * k + 1];
  }
  if (rc != ORC_OK) {
    free(cell);
    free(ncell);
    free(sv);
    return rc;
  }
  double *vs = (double *)calloc((size_t)(2 * C), sizeof(double));
  ORC_CELLS_PARALLEL
  for (int64_t c = 0; c < C; ++c)
    if (ncell[c] > 0) { /* Eq. 8; an empty cell keeps v_s = 0 (R8) */
      vs[2 * c] = sv[2 * c] / ncell[c];
      vs[2 * c + 1] = sv[2 * c + 1] / ncell[c];
    }

  /* ---- 3) collision and streaming ---- */
  double *fstar = (double *)malloc((size_t)(9 * C) * sizeof(double));
  double *rho = (double *)malloc((size_t)C * sizeof(double));
  double *ug = (double *)malloc((size_t)(2 * C) * sizeof(double));
  double *fpg = (double *)malloc((size_t)(2 * C) * sizeof(double));
  double *beta = (double *)malloc((size_t)C * sizeof(double));
  ORC_CELLS_PARALLEL
  for (int64_t c = 0; c < C; ++c) {
    double fl[9], fs[9], o[8];
    for (int i = 0; i < 9; ++i) fl[i] = f[i * C + c];
    orc_collide_node(p, fl, ncell[c], vs + 2 * c, fs, o);
    for (int i = 0; i < 9; ++i) fstar[i * C + c] = fs[i];
    rho[c] = o[0];
    ug[2 * c] = o[1];
    ug[2 * c + 1] = o[2];
    fpg[2 * c] = o[3];
    fpg[2 * c + 1] = o[4];
    beta[c] = o[5];
  }
  orc_stream(p, inlet_uy, fstar, f);
  free(fstar);

  /* ---- 4) drag ---- */
  double *pres = (double *)malloc((size_t)C * sizeof(double));
  double *grad = (double *)malloc((size_t)(2 * C) * sizeof(double));
  double *es3 = (double *)malloc((size_t)C * sizeof(double));
  double *ugx = (double *)malloc((size_t)C * sizeof(double));
  double *ugy = (double *)malloc((size_t)C * sizeof(double));
  double *gx = (double *)malloc((size_t)C * sizeof(double));
  double *gy = (double *)malloc((size_t)C * sizeof(double));
  ORC_CELLS_PARALLEL
  for (int64_t c = 0; c < C; ++c) {
    double pr[6];
    orc_cell_props(p, ncell[c], pr);
    es3[c] = pr[2];
    pres[c] = rho[c] / 3.0;
    ugx[c] = ug[2 * c];
    ugy[c] = ug[2 * c + 1];
  }
  orc_grad_p(p, pres, grad);
  ORC_CELLS_PARALLEL
  for (int64_t c = 0; c < C; ++c) {
    gx[c] = grad[2 * c];
    gy[c] = grad[2 * c + 1];
  }
  double vp = vol_p(p);
  double *fpre = (double *)malloc(NP * 2 * sizeof(double));
  double *gpk = (double *)malloc(NP * 2 * sizeof(double));
  double *fd = (double *)malloc(NP * 2 * sizeof(double));
  double *fcell = (double *)calloc((size_t)(2 * C), sizeof(double));
  double *acell = (double *)calloc((size_t)(2 * C), sizeof(double)); /* sum of |F_pre| */
  for (int64_t k = 0; k < np; ++k) {
    double px = pos[2 * k], py = pos[2 * k + 1];
    double uk_x = orc_interp(p, ugx, px, py);
    double uk_y = orc_interp(p, ugy, px, py);
    if (out && out->upart) {
      out->upart[2 * k] = uk_x;
      out->upart[2 * k + 1] = uk_y;
    }
    double ek = orc_interp(p, es3, px, py); /* solid fraction 1 - eps_k (R13) */
    double bk = orc_interp(p, beta, px, py);
    gpk[2 * k] = orc_interp(p, gx, px, py);
    gpk[2 * k + 1] = orc_interp(p, gy, px, py);
    /* Eq. 26 */
    fpre[2 * k] = vp * bk / ek * (uk_x - vel[2 * k]);
    fpre[2 * k + 1] = vp * bk / ek * (uk_y - vel[2 * k + 1]);
    /* Eq. 27, summed in ascending particle index */
    fcell[2 * cell[k]] += fpre[2 * k];
    fcell[2 * cell[k] + 1] += fpre[2 * k + 1];
    acell[2 * cell[k]] += fabs(fpre[2 * k]);
    acell[2 * cell[k] + 1] += fabs(fpre[2 * k + 1]);
  }
  /* R49 (mode 2): where the cell's pre-drags cancel, sum |F_pre| beyond
   * ORC_CANCEL_MAX times |sum F_pre|, the denominator is taken as zero. */
  if (p->drag_ratio_mode == 2)
    for (int64_t c = 0; c < 2 * C; ++c)
      if (acell[c] > ORC_CANCEL_MAX * fabs(fcell[c])) fcell[c] = 0.0;
  int64_t nzero = 0;
  for (int64_t c = 0; c < C; ++c)
    for (int a = 0; a < 2; ++a)
      if (ncell[c] > 0 && fcell[2 * c + a] == 0.0) ++nzero;
  /* Eq. 28: signed ratio (R15) or literal absolute values; a zero
   * denominator splits F_p->g equally (R16). */
  for (int64_t k = 0; k < np; ++k) {
    int32_t c = cell[k];
    for (int a = 0; a < 2; ++a) {
      double den = fcell[2 * c + a], fg = fpg[2 * c + a];
      double v;
      if (den == 0.0)
        v = -fg / ncell[c];
      else if (p->drag_ratio_mode == 1)
        v = fabs(fg) / fabs(den) * fpre[2 * k + a];
      else
        v = -fg * fpre[2 * k + a] / den;
      fd[2 * k + a] = v;
    }
  }

  /* ---- 5) and 6): integration, then contacts at the new positions,
   * collisions and walls, once per sub-step (R41) ---- */
  const int nsub = p->n_sub > 1 ? p->n_sub : 1;
  const double h = 1.0 / (double)nsub;
  double *acc = (double *)malloc(NP * 2 * sizeof(double));
  accelerations(p, np, fd, gpk, acc);
  int64_t cap = out && out->pairs ? out->pair_cap : 0;
  int64_t cap_eff = cap > 0 ? cap : (np * 16 + 16);
  int32_t *pairs = out && out->pairs ? out->pairs : (int32_t *)malloc((size_t)cap_eff * 2 * sizeof(int32_t));
  int64_t npairs = 0, ncoll = 0, nwall = 0, ncross = 0;
  for (int sub = 0; sub < nsub && rc == ORC_OK; ++sub) {
    ncross += advance(p, np, pos, vel, acc, h);
    npairs = ncoll = nwall = 0;
    rc = orc_contacts_cells(p, np, pos, pairs, cap_eff, &npairs);
    if (rc == ORC_OK) {
      orc_resolve(p, np, pos, vel, pairs, npairs, &ncoll);
      orc_walls(p, np, pos, vel, &nwall);
    }
  }

  if (out) {
    if (out->ncell) memcpy(out->ncell, ncell, (size_t)C * sizeof(int32_t));
    if (out->vs) memcpy(out->vs, vs, (size_t)(2 * C) * sizeof(double));
    if (out->rho) memcpy(out->rho, rho, (size_t)C * sizeof(double));
    if (out->ugas) memcpy(out->ugas, ug, (size_t)(2 * C) * sizeof(double));
    if (out->fpg) memcpy(out->fpg, fpg, (size_t)(2 * C) * sizeof(double));
    if (out->beta) memcpy(out->beta, beta, (size_t)C * sizeof(double));
    if (out->fd && np > 0) memcpy(out->fd, fd, NP * 2 * sizeof(double));
    if (out->fpre && np > 0) memcpy(out->fpre, fpre, NP * 2 * sizeof(double));
    if (out->acc && np > 0) memcpy(out->acc, acc, NP * 2 * sizeof(double));
    out->npairs = npairs;
    out->ncollisions = ncoll;
    out->nwall = nwall;
    out->nzero_den = nzero;
    out->ncross = ncross;
  }
  if (!(out && out->pairs)) free(pairs);
  free(acc);
  free(cell);
  free(ncell);
  free(sv);
  free(vs);
  free(rho);
  free(ug);
  free(fpg);
  free(beta);
  free(pres);
  free(grad);
  free(es3);
  free(ugx);
  free(ugy);
  free(gx);
  free(gy);
  free(fpre);
  free(gpk);
  free(fd);
  free(acell);
  free(fcell);
  return rc;
}

/* Global sums for the conservation checks: out[0] mass sum f, out[1..2] fluid
 * momentum sum c f, out[3..4] particle momentum sum m v.  Plain sequential sums. */
void orc_conservation(const orc_params *p, const double *f, int64_t np, const double *vel, double *out) {
  const int64_t C = (int64_t)p->nx * p->ny;
  double mass = 0.0, px = 0.0, py = 0.0, qx = 0.0, qy = 0.0;
  for (int64_t c = 0; c < C; ++c)
    for (int i = 0; i < 9; ++i) {
      double v = f[i * C + c];
      mass += v;
      px += CX[i] * v;
      py += CY[i] * v;
    }
  double m = mass_p(p);
  for (int64_t k = 0; k < np; ++k) {
    qx += m * vel[2 * k];
    qy += m * vel[2 * k + 1];
  }
  out[0] = mass;
  out[1] = px;
  out[2] = py;
  out[3] = qx;
  out[4] = qy;
}

/* ==== 3-D gas lattice (the 3-D extension the paper names as future work) ====
 * D3Q19: the rest velocity, the 6 face neighbours (weight 1/18) and the 12
 * edge neighbours (weight 1/36), rest weight 1/3, c_s^2 = 1/3; the
 * equilibrium has the same second-order form as in 2-D (Eq. 4 with
 * c_i.u in three dimensions).  Only the gas part is here: the BGK step on a
 * fully periodic box, the first piece of the 3-D coupled step. */
static const int C3[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
                              {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
                              {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

static double w3(int i) { return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }

void orc3_lattice(int32_t *c, double *w) {
  for (int i = 0; i < 19; ++i) {
    for (int a = 0; a < 3; ++a) c[3 * i + a] = C3[i][a];
    w[i] = w3(i);
  }
}

double orc3_feq(int i, double rho, double ux, double uy, double uz) {
  double cu = C3[i][0] * ux + C3[i][1] * uy + C3[i][2] * uz;
  double uu = ux * ux + uy * uy + uz * uz;
  return w3(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
}

/*
 * One BGK step on a periodic nx x ny x nz box (Eqs. 2-3 on the 3-D lattice):
 * moments, relaxation towards f^eq with 1/tau, then pull streaming
 * f_i(x) <- f*_i(x - c_i).  f[19][nz][ny][nx] is advanced in place.
 */
void orc3_bgk_step(int32_t nx, int32_t ny, int32_t nz, double tau, double *f) {
  const int64_t C = (int64_t)nx * ny * nz;
  double *fs = (double *)malloc((size_t)(19 * C) * sizeof(double));
  for (int64_t c = 0; c < C; ++c) {
    double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    for (int i = 0; i < 19; ++i) {
      double v = f[i * C + c];
      rho += v;
      jx += C3[i][0] * v;
      jy += C3[i][1] * v;
      jz += C3[i][2] * v;
    }
    double ux = jx / rho, uy = jy / rho, uz = jz / rho;
    for (int i = 0; i < 19; ++i) {
      double v = f[i * C + c];
      fs[i * C + c] = v - (v - orc3_feq(i, rho, ux, uy, uz)) / tau;
    }
  }
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int64_t c = ((int64_t)z * ny + y) * nx + x;
        for (int i = 0; i < 19; ++i) {
          int sx = ((x - C3[i][0]) % nx + nx) % nx;
          int sy = ((y - C3[i][1]) % ny + ny) % ny;
          int sz = ((z - C3[i][2]) % nz + nz) % nz;
          f[i * C + c] = fs[i * C + ((int64_t)sz * ny + sy) * nx + sx];
        }
      }
  free(fs);
}

/* The opposite of each D3Q19 direction, found by search so that no table has
 * to be trusted. */
static int opp3(int i) {
  for (int k = 0; k < 19; ++k)
    if (C3[k][0] == -C3[i][0] && C3[k][1] == -C3[i][1] && C3[k][2] == -C3[i][2]) return k;
  return -1;
}

/*
 * One partially-saturated step of the 3-D gas lattice with given solids
 * (the 2-D collision of Eqs. 6-7 and the force of Eq. 25 on D3Q19; R45):
 * cell c holds n[c] spheres of diameter d (lattice units) moving with mean
 * velocity vs[a][c].  Solid fraction eps_s = n pi d^3 / 6, at most the
 * densest sphere packing pi / (3 sqrt 2); gamma from Eq. 9 at eps_s;
 *   Om_i  = f_opp(i) - f_i + f^eq_i(rho, v_s) - f^eq_opp(i)(rho, u)   (Eq. 7)
 *   f*_i  = f_i - (1 - gamma) / tau (f_i - f^eq_i(rho, u)) + gamma Om_i
 *   F     = gamma sum_i c_i Om_i                                      (Eq. 25)
 * then pull streaming on the periodic box.  f[19][nz][ny][nx] is advanced
 * in place; force[3][nz][ny][nx] receives F (the momentum the solids give
 * the gas in this step).
 */
void orc3_psm_step(int32_t nx, int32_t ny, int32_t nz, double tau, double d, const int32_t *n,
                   const double *vs, double *f, double *force) {
  const int64_t C = (int64_t)nx * ny * nz;
  const double vol = PI * d * d * d / 6.0;
  const double cap = PI / (3.0 * sqrt(2.0));
  double *fs = (double *)malloc((size_t)(19 * C) * sizeof(double));
  for (int64_t c = 0; c < C; ++c) {
    double es = (double)n[c] * vol;
    if (es > cap) es = cap;
    double gam = orc_gamma(es, tau);
    double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    for (int i = 0; i < 19; ++i) {
      double v = f[i * C + c];
      rho += v;
      jx += C3[i][0] * v;
      jy += C3[i][1] * v;
      jz += C3[i][2] * v;
    }
    double ux = jx / rho, uy = jy / rho, uz = jz / rho;
    double vx = vs[c], vy = vs[C + c], vz = vs[2 * C + c];
    double fx = 0.0, fy = 0.0, fz = 0.0;
    for (int i = 0; i < 19; ++i) {
      int o = opp3(i);
      double fi = f[i * C + c];
      double om = f[o * C + c] - fi + orc3_feq(i, rho, vx, vy, vz) - orc3_feq(o, rho, ux, uy, uz);
      fs[i * C + c] = fi - (1.0 - gam) / tau * (fi - orc3_feq(i, rho, ux, uy, uz)) + gam * om;
      fx += C3[i][0] * om;
      fy += C3[i][1] * om;
      fz += C3[i][2] * om;
    }
    force[c] = gam * fx;
    force[C + c] = gam * fy;
    force[2 * C + c] = gam * fz;
  }
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int64_t c = ((int64_t)z * ny + y) * nx + x;
        for (int i = 0; i < 19; ++i) {
          int sx = ((x - C3[i][0]) % nx + nx) % nx;
          int sy = ((y - C3[i][1]) % ny + ny) % ny;
          int sz = ((z - C3[i][2]) % nz + nz) % nz;
          f[i * C + c] = fs[i * C + ((int64_t)sz * ny + sy) * nx + sx];
        }
      }
  free(fs);
}

/* ==== the 3-D coupled step (the fully 3-D simulation the paper names as the
 * natural extension, Sec. 4) ====
 * The procedure of Sec. 2.4 on a fully periodic D3Q19 box with spheres of
 * diameter d (R48):
 *   2) per cell: n (Eq. 8's count), v_s (Eq. 8, ascending index), the solid
 *      fraction eps_s = min(n pi d^3 / 6, pi / (3 sqrt 2)) (R45), the voidage
 *      eps_g = 1 - eps_s, gamma (Eq. 9 at eps_s), omega (Eq. 20 at eps_g, or
 *      omega_dense where eps_g <= 0.74);
 *   3) Eq. 23 with the solid term of Eq. 7 on D3Q19 and the body-force source
 *      3 w_i c_i.G; F_pg = omega gamma sum c_i Om_i (Eq. 25); the superficial
 *      velocity of Eq. 24 with G/2, the actual gas velocity u_sup / eps_g; beta
 *      of Eqs. 19, 21, 22 at eps_g with the slip |u_gas - v_s|; p = rho / 3;
 *      pull streaming on the periodic box;
 *   4) trilinear interpolation (nodes at the cell centres, s = P - 1/2) of
 *      u_gas, eps_s, beta and grad p (central differences of p); F_pre of
 *      Eq. 26, the cell sums of Eq. 27 in ascending index, Eq. 28 signed with
 *      the equal split of a zero denominator (R15, R16);
 *   5) v <- v + g_eff + (F_d - V_p grad p_k) / m, P <- P + v, periodic wrap;
 *   6) contacts |P_i - P_j|^2 <= d^2 (minimum image, i < j), binary
 *      collisions of Eqs. 17-18 in lexicographic order.
 */
typedef struct {
  int32_t nx, ny, nz;
  double tau, rho_g, rho_s, d, e_pp;
  double g[3];  /* gravity on particles, before the (1 - rho_g/rho_s) factor */
  double G[3];  /* body force on the gas per cell */
  double omega_dense;
  int32_t pressure_sign; /* -1 physical (R17), 0 off */
} orc3_params;

typedef struct {
  int32_t *ncell; /* [C] */
  double *vs;     /* [C][3] */
  double *rho;    /* [C] */
  double *ugas;   /* [C][3] */
  double *fpg;    /* [C][3] */
  double *beta;   /* [C] */
  double *fd;     /* [N][3] */
  double *acc;    /* [N][3] acceleration of Eq. 16 */
  int32_t *pairs; /* [cap][2] */
  int64_t pair_cap;
  int64_t npairs, ncollisions; /* out */
} orc3_out;

static int64_t cell3(const orc3_params *p, int x, int y, int z) {
  return ((int64_t)z * p->ny + y) * p->nx + x;
}
static int wrap_i3(int i, int n) { return ((i % n) + n) % n; }

/* Per-count cell quantities in 3-D: out[0] eps_s, out[1] eps_g, out[2] gamma,
 * out[3] omega. */
void orc3_cell_props(const orc3_params *p, int64_t n, double *out) {
  double es = (double)n * (PI * p->d * p->d * p->d / 6.0);
  double cap = PI / (3.0 * sqrt(2.0));
  if (es > cap) es = cap;
  double eg = 1.0 - es;
  out[0] = es;
  out[1] = eg;
  out[2] = orc_gamma(es, p->tau);
  out[3] = eg > 0.74 ? orc_omega_emms(eg) : p->omega_dense;
}

/* Trilinear stencil on the periodic box: the 8 nodes around P (node (i,j,k)
 * at the cell centre) and their weights. */
void orc3_stencil(const orc3_params *p, const double *P, int64_t *idx, double *wt) {
  double s[3], t[3];
  int i0[3];
  const int n[3] = {p->nx, p->ny, p->nz};
  for (int a = 0; a < 3; ++a) {
    s[a] = P[a] - 0.5;
    double fl = floor(s[a]);
    t[a] = s[a] - fl;
    i0[a] = (int)fl;
  }
  for (int q = 0; q < 8; ++q) {
    int ox = q & 1, oy = (q >> 1) & 1, oz = q >> 2;
    idx[q] = cell3(p, wrap_i3(i0[0] + ox, n[0]), wrap_i3(i0[1] + oy, n[1]), wrap_i3(i0[2] + oz, n[2]));
    wt[q] = (ox ? t[0] : 1.0 - t[0]) * (oy ? t[1] : 1.0 - t[1]) * (oz ? t[2] : 1.0 - t[2]);
  }
}

double orc3_interp(const orc3_params *p, const double *q, const double *P) {
  int64_t idx[8];
  double wt[8];
  orc3_stencil(p, P, idx, wt);
  double v = 0.0;
  for (int k = 0; k < 8; ++k) v += wt[k] * q[idx[k]];
  return v;
}

static void sep3(const orc3_params *p, const double *a, const double *b, double *d) {
  const int n[3] = {p->nx, p->ny, p->nz};
  for (int k = 0; k < 3; ++k) {
    double x = a[k] - b[k];
    if (x > 0.5 * n[k])
      x -= n[k];
    else if (x < -0.5 * n[k])
      x += n[k];
    d[k] = x;
  }
}

static int in_contact3(const orc3_params *p, const double *a, const double *b) {
  double d[3];
  sep3(p, a, b, d);
  return d[0] * d[0] + d[1] * d[1] + d[2] * d[2] <= p->d * p->d;
}

int orc3_contacts_brute(const orc3_params *p, int64_t np, const double *pos, int32_t *pairs, int64_t cap,
                        int64_t *npairs) {
  int64_t m = 0;
  for (int64_t i = 0; i < np; ++i)
    for (int64_t j = i + 1; j < np; ++j)
      if (in_contact3(p, pos + 3 * i, pos + 3 * j)) {
        if (m >= cap) {
          *npairs = m;
          return ORC_E_CAPACITY;
        }
        pairs[2 * m] = (int32_t)i;
        pairs[2 * m + 1] = (int32_t)j;
        ++m;
      }
  *npairs = m;
  return ORC_OK;
}

/* The same set through 1-cell bins: a partner lies in one of the 27 cells
 * around a particle (d < 1); lexicographic order. */
int orc3_contacts_cells(const orc3_params *p, int64_t np, const double *pos, int32_t *pairs, int64_t cap,
                        int64_t *npairs) {
  const int64_t C = (int64_t)p->nx * p->ny * p->nz;
  int32_t *cell = (int32_t *)malloc((size_t)(np > 0 ? np : 1) * sizeof(int32_t));
  int64_t *start = (int64_t *)malloc((size_t)(C + 1) * sizeof(int64_t));
  int64_t *list = (int64_t *)malloc((size_t)(np > 0 ? np : 1) * sizeof(int64_t));
  for (int64_t k = 0; k < np; ++k)
    cell[k] = (int32_t)cell3(p, (int)floor(pos[3 * k]), (int)floor(pos[3 * k + 1]), (int)floor(pos[3 * k + 2]));
  bucket(C, np, cell, start, list);
  int64_t m = 0;
  int rc = ORC_OK;
  for (int64_t i = 0; i < np && rc == ORC_OK; ++i) {
    int cx = (int)floor(pos[3 * i]), cy = (int)floor(pos[3 * i + 1]), cz = (int)floor(pos[3 * i + 2]);
    /* distinct neighbour cells only (a box narrower than 3 cells repeats them) */
    int64_t seen[27];
    int nseen = 0;
    for (int oz = -1; oz <= 1; ++oz)
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
          int64_t c = cell3(p, wrap_i3(cx + ox, p->nx), wrap_i3(cy + oy, p->ny), wrap_i3(cz + oz, p->nz));
          int dup = 0;
          for (int q = 0; q < nseen; ++q) dup |= seen[q] == c;
          if (dup) continue;
          seen[nseen++] = c;
          for (int64_t s = start[c]; s < start[c + 1] && rc == ORC_OK; ++s) {
            int64_t j = list[s];
            if (j <= i || !in_contact3(p, pos + 3 * i, pos + 3 * j)) continue;
            if (m >= cap) {
              rc = ORC_E_CAPACITY;
              break;
            }
            pairs[2 * m] = (int32_t)i;
            pairs[2 * m + 1] = (int32_t)j;
            ++m;
          }
        }
  }
  qsort(pairs, (size_t)m, 2 * sizeof(int32_t), cmp_pair);
  *npairs = m;
  free(cell);
  free(start);
  free(list);
  return rc;
}

/* Eqs. 17-18 for spheres in 3-D over the pairs in order, current velocities;
 * a pair collides only if (P_1 - P_2).(v_1 - v_2) < 0. */
void orc3_resolve(const orc3_params *p, const double *pos, double *vel, const int32_t *pairs, int64_t npairs,
                  int64_t *ncoll) {
  double m1 = p->rho_s * (PI * p->d * p->d * p->d / 6.0), m2 = m1; /* m = rho_s V_p (R19) */
  int64_t nc = 0;
  for (int64_t q = 0; q < npairs; ++q) {
    int64_t i = pairs[2 * q], j = pairs[2 * q + 1];
    double d[3];
    sep3(p, pos + 3 * i, pos + 3 * j, d);
    double dv[3] = {vel[3 * i] - vel[3 * j], vel[3 * i + 1] - vel[3 * j + 1], vel[3 * i + 2] - vel[3 * j + 2]};
    double dot = dv[0] * d[0] + dv[1] * d[1] + dv[2] * d[2];
    if (!(dot < 0.0)) continue;
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double q0 = (1.0 + p->e_pp) * dot / r2;
    double ci = q0 * m2 / (m1 + m2), cj = q0 * m1 / (m1 + m2);
    for (int a = 0; a < 3; ++a) {
      vel[3 * i + a] = vel[3 * i + a] - ci * d[a];
      vel[3 * j + a] = vel[3 * j + a] + cj * d[a];
    }
    ++nc;
  }
  if (ncoll) *ncoll = nc;
}

static double wrap3(double x, double L) {
  if (x >= L) {
    x -= L;
  } else if (x < 0.0) {
    x += L;
    if (x >= L) x = 0.0;
  }
  return x;
}

int orc3_step(const orc3_params *p, double *f, int64_t np, double *pos, double *vel, orc3_out *out) {
  const int nx = p->nx, ny = p->ny, nz = p->nz;
  const int64_t C = (int64_t)nx * ny * nz;
  const size_t NP = (size_t)(np > 0 ? np : 1);
  const double vp = PI * p->d * p->d * p->d / 6.0, m = p->rho_s * vp;
  const double mu = p->rho_g * ((p->tau - 0.5) / 3.0);
  /* ---- 2) deposition ---- */
  int32_t *cell = (int32_t *)malloc(NP * sizeof(int32_t));
  int32_t *ncell = (int32_t *)calloc((size_t)C, sizeof(int32_t));
  double *vs = (double *)calloc((size_t)(3 * C), sizeof(double));
  for (int64_t k = 0; k < np; ++k) {
    int ix = (int)floor(pos[3 * k]), iy = (int)floor(pos[3 * k + 1]), iz = (int)floor(pos[3 * k + 2]);
    if (ix < 0 || ix >= nx || iy < 0 || iy >= ny || iz < 0 || iz >= nz) {
      free(cell);
      free(ncell);
      free(vs);
      return ORC_E_DOMAIN;
    }
    int64_t c = cell3(p, ix, iy, iz);
    cell[k] = (int32_t)c;
    ncell[c] += 1;
    for (int a = 0; a < 3; ++a) vs[3 * c + a] += vel[3 * k + a];
  }
  for (int64_t c = 0; c < C; ++c)
    if (ncell[c] > 0)
      for (int a = 0; a < 3; ++a) vs[3 * c + a] = vs[3 * c + a] / ncell[c];
  /* ---- 3) collision and streaming ---- */
  double *fs = (double *)malloc((size_t)(19 * C) * sizeof(double));
  double *rho = (double *)malloc((size_t)C * sizeof(double));
  double *ug = (double *)malloc((size_t)(3 * C) * sizeof(double));
  double *fpg = (double *)malloc((size_t)(3 * C) * sizeof(double));
  double *beta = (double *)malloc((size_t)C * sizeof(double));
  double *es = (double *)malloc((size_t)C * sizeof(double));
  orc_params bp; /* the drag law's parameters (orc_beta) */
  memset(&bp, 0, sizeof bp);
  bp.tau = p->tau;
  bp.rho_g = p->rho_g;
  bp.d = p->d;
  ORC_CELLS_PARALLEL
  for (int64_t c = 0; c < C; ++c) {
    double pr[4];
    orc3_cell_props(p, ncell[c], pr);
    const double gam = pr[2], omg = pr[3] * pr[2];
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 19; ++i) {
      double v = f[i * C + c];
      r += v;
      for (int a = 0; a < 3; ++a) j[a] += C3[i][a] * v;
    }
    double u[3] = {j[0] / r, j[1] / r, j[2] / r};
    const double *v = vs + 3 * c;
    double F[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < 19; ++i) {
      int o = opp3(i);
      double fi = f[i * C + c];
      double om = f[o * C + c] - fi + orc3_feq(i, r, v[0], v[1], v[2]) - orc3_feq(o, r, u[0], u[1], u[2]);
      double src = 3.0 * w3(i) * (C3[i][0] * p->G[0] + C3[i][1] * p->G[1] + C3[i][2] * p->G[2]);
      fs[i * C + c] = fi - (1.0 - gam) / p->tau * (fi - orc3_feq(i, r, u[0], u[1], u[2])) + omg * om + src;
      for (int a = 0; a < 3; ++a) F[a] += C3[i][a] * om;
    }
    double sl2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      fpg[3 * c + a] = omg * F[a];
      double usup = (j[a] + 0.5 * fpg[3 * c + a] + 0.5 * p->G[a]) / r;
      ug[3 * c + a] = usup / pr[1];
      double dd = ug[3 * c + a] - v[a];
      sl2 += dd * dd;
    }
    rho[c] = r;
    es[c] = pr[0];
    beta[c] = orc_beta(&bp, pr[1], pr[3], sqrt(sl2));
  }
  ORC_CELLS_PARALLEL
  for (int64_t c = 0; c < C; ++c) {
    int x = (int)(c % nx), y = (int)((c / nx) % ny), z = (int)(c / ((int64_t)nx * ny));
    for (int i = 0; i < 19; ++i)
      f[i * C + c] = fs[i * C + cell3(p, wrap_i3(x - C3[i][0], nx), wrap_i3(y - C3[i][1], ny),
                                       wrap_i3(z - C3[i][2], nz))];
  }
  free(fs);
  /* ---- 4) drag ---- */
  double *gp = (double *)malloc((size_t)(3 * C) * sizeof(double));
  ORC_CELLS_PARALLEL
  for (int64_t c = 0; c < C; ++c) {
    int x = (int)(c % nx), y = (int)((c / nx) % ny), z = (int)(c / ((int64_t)nx * ny));
    gp[3 * c] = (rho[cell3(p, wrap_i3(x + 1, nx), y, z)] / 3.0 - rho[cell3(p, wrap_i3(x - 1, nx), y, z)] / 3.0) * 0.5;
    gp[3 * c + 1] = (rho[cell3(p, x, wrap_i3(y + 1, ny), z)] / 3.0 - rho[cell3(p, x, wrap_i3(y - 1, ny), z)] / 3.0) * 0.5;
    gp[3 * c + 2] = (rho[cell3(p, x, y, wrap_i3(z + 1, nz))] / 3.0 - rho[cell3(p, x, y, wrap_i3(z - 1, nz))] / 3.0) * 0.5;
  }
  double *comp = (double *)malloc((size_t)C * sizeof(double));
  double *fpre = (double *)malloc(NP * 3 * sizeof(double));
  double *gpk = (double *)malloc(NP * 3 * sizeof(double));
  double *fcell = (double *)calloc((size_t)(3 * C), sizeof(double));
  double *uk = (double *)malloc(NP * 3 * sizeof(double));
  double *ek = (double *)malloc(NP * sizeof(double));
  double *bk = (double *)malloc(NP * sizeof(double));
  for (int a = 0; a < 3; ++a) {
    for (int64_t c = 0; c < C; ++c) comp[c] = ug[3 * c + a];
    for (int64_t k = 0; k < np; ++k) uk[3 * k + a] = orc3_interp(p, comp, pos + 3 * k);
    for (int64_t c = 0; c < C; ++c) comp[c] = gp[3 * c + a];
    for (int64_t k = 0; k < np; ++k) gpk[3 * k + a] = orc3_interp(p, comp, pos + 3 * k);
  }
  for (int64_t k = 0; k < np; ++k) {
    ek[k] = orc3_interp(p, es, pos + 3 * k);
    bk[k] = orc3_interp(p, beta, pos + 3 * k);
  }
  for (int64_t k = 0; k < np; ++k)
    for (int a = 0; a < 3; ++a) {
      fpre[3 * k + a] = vp * bk[k] / ek[k] * (uk[3 * k + a] - vel[3 * k + a]); /* Eq. 26 */
      fcell[3 * cell[k] + a] += fpre[3 * k + a];                                /* Eq. 27 */
    }
  double *fd = (double *)malloc(NP * 3 * sizeof(double));
  double *acc = (double *)malloc(NP * 3 * sizeof(double));
  const double sgn = (double)p->pressure_sign; /* pressure force s V_p grad p, s = -1 (R17) */
  for (int64_t k = 0; k < np; ++k)
    for (int a = 0; a < 3; ++a) {
      int32_t c = cell[k];
      double den = fcell[3 * c + a], fg = fpg[3 * c + a];
      fd[3 * k + a] = den == 0.0 ? -fg / ncell[c] : -fg * fpre[3 * k + a] / den; /* Eq. 28 */
      double geff = (1.0 - p->rho_g / p->rho_s) * p->g[a];
      acc[3 * k + a] = geff + (fd[3 * k + a] + sgn * vp * gpk[3 * k + a]) / m;
    }
  /* ---- 5) integration ---- */
  const double L[3] = {nx, ny, nz};
  for (int64_t k = 0; k < np; ++k)
    for (int a = 0; a < 3; ++a) {
      vel[3 * k + a] = vel[3 * k + a] + acc[3 * k + a];
      pos[3 * k + a] = wrap3(pos[3 * k + a] + vel[3 * k + a], L[a]);
    }
  /* ---- 6) contacts and collisions ---- */
  int64_t cap = out && out->pairs ? out->pair_cap : 0;
  int64_t cap_eff = cap > 0 ? cap : (np * 32 + 16);
  int32_t *pairs = out && out->pairs ? out->pairs : (int32_t *)malloc((size_t)cap_eff * 2 * sizeof(int32_t));
  int64_t npairs = 0, ncoll = 0;
  int rc = orc3_contacts_cells(p, np, pos, pairs, cap_eff, &npairs);
  if (rc == ORC_OK) orc3_resolve(p, pos, vel, pairs, npairs, &ncoll);
  if (out) {
    if (out->ncell) memcpy(out->ncell, ncell, (size_t)C * sizeof(int32_t));
    if (out->vs) memcpy(out->vs, vs, (size_t)(3 * C) * sizeof(double));
    if (out->rho) memcpy(out->rho, rho, (size_t)C * sizeof(double));
    if (out->ugas) memcpy(out->ugas, ug, (size_t)(3 * C) * sizeof(double));
    if (out->fpg) memcpy(out->fpg, fpg, (size_t)(3 * C) * sizeof(double));
    if (out->beta) memcpy(out->beta, beta, (size_t)C * sizeof(double));
    if (out->fd && np > 0) memcpy(out->fd, fd, NP * 3 * sizeof(double));
    if (out->acc && np > 0) memcpy(out->acc, acc, NP * 3 * sizeof(double));
    out->npairs = npairs;
    out->ncollisions = ncoll;
  }
  if (!(out && out->pairs)) free(pairs);
  free(cell);
  free(ncell);
  free(vs);
  free(rho);
  free(ug);
  free(fpg);
  free(beta);
  free(es);
  free(gp);
  free(comp);
  free(fpre);
  free(gpk);
  free(fcell);
  free(uk);
  free(ek);
  free(bk);
  free(fd);
  free(acc);
  return rc;
}

/* FP64 conservation sums of the 3-D state: out[0] mass, out[1..3] gas
 * momentum, out[4..6] particle momentum. */
void orc3_conservation(const orc3_params *p, const double *f, int64_t np, const double *vel, double *out) {
  const int64_t C = (int64_t)p->nx * p->ny * p->nz;
  const double m = p->rho_s * (PI * p->d * p->d * p->d / 6.0);
  for (int k = 0; k < 7; ++k) out[k] = 0.0;
  for (int64_t c = 0; c < C; ++c)
    for (int i = 0; i < 19; ++i) {
      double v = f[i * C + c];
      out[0] += v;
      for (int a = 0; a < 3; ++a) out[1 + a] += C3[i][a] * v;
    }
  for (int64_t k = 0; k < np; ++k)
    for (int a = 0; a < 3; ++a) out[4 + a] += m * vel[3 * k + a];
}
