/*
 * smc_oracle.c -- plain FP64 CPU oracle for the checkerboard single-spin-flip
 * Metropolis chain of nearest-neighbour O(n) spin models (Weigel & Yavors'kii,
 * "GPU accelerated Monte Carlo simulations of lattice spin models", Sec. 2).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or constant generator
 * with the HIP path.  It is deliberately slow and literal:
 *   - spins are stored in natural site order i = x + L*y + L*L*z;
 *   - every site recomputes its neighbours' indices with mod arithmetic;
 *   - every Ising attempt draws the full 32-bit uniform (prefix byte plus the
 *     24-bit refinement word), even though the byte alone decides 255/256 of
 *     the uphill attempts;
 *   - all floating point is double precision (continuous spins, couplings,
 *     energies); FP32 inputs are promoted exactly.
 *
 * What it computes (paper references are to the sections/equations of the
 * paper above):
 *   Eq. (1)  H = -sum_<ij> J_ij s_i . s_j on periodic square (d=2) or simple
 *            cubic (d=3) lattices, n = 1 (Ising), 2 (XY), 3 (Heisenberg).
 *   Eq. (2)  p_acc = min[1, exp(-beta dE)] for single-spin moves.
 *   Sec. 2   checkerboard decomposition: all sites of one sublattice (colour)
 *            are updated from the same configuration of the other colour, then
 *            the other colour is treated the same way; tabulated Boltzmann
 *            factors for the discrete Ising energy changes; aggregate
 *            quantities (energy, magnetisation) accumulated in double.
 *
 * Random numbers (the paper uses one 32-bit LCG per thread; here a stateless
 * counter-based generator keyed by seed, sweep and site, so that any parallel
 * schedule reproduces the same chain) come from Philox4x32-10 as published by
 * Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3"
 * (SC'11).  The assignment of counter words, tags, words and bytes to sites is
 * the project's RNG contract; it is written out again independently on the
 * GPU side.
 *
 * Readings of the paper that this file fixes (listed in the design notes):
 * periodic boundaries, L even, colour c = (x+y+z) mod 2, colour 0 first,
 * strict comparison u < p with dE <= 0 always accepted, forward-bond energy
 * with each bond counted once, L = 2 allowed here (the +mu and -mu neighbour
 * coincide and both bond terms are counted).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11).                                    */
/* A round multiplies counter words 0 and 2 by two fixed odd multipliers    */
/* (full 64-bit products), and forms the next counter from the high halves  */
/* xored with the remaining counter words and the round key, and from the   */
/* low halves.  The key is advanced by the two Weyl increments after every  */
/* round.  Ten rounds.                                                      */
/* ------------------------------------------------------------------------ */
static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u;
static const uint32_t PHILOX_W1 = 0xBB67AE85u;

ORACLE_API void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                                     uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += PHILOX_W0;
    k1 += PHILOX_W1;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* RNG contract: key = seed split in two 32-bit halves, counter =
 * (block, sweep-or-axis, replica, tag) with tag = colour | (purpose << 1). */
enum {
  PURPOSE_ISING_PREFIX = 0,
  PURPOSE_ISING_REFINE = 1,
  PURPOSE_CONTINUOUS = 2,
  PURPOSE_INIT_SPIN = 3,
  PURPOSE_COUPLING = 4
};

static void draw(uint64_t seed, uint32_t block, uint32_t w1, uint32_t replica,
                 uint32_t tag, uint32_t out[4]) {
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  uint32_t ctr[4] = {block, w1, replica, tag};
  oracle_philox4x32_10(ctr, key, out);
}

/* Uniform on (0,1): the top 23 bits of a word, centred in their cell.  The
 * value (2k+1)/2^24 has at most 24 significant bits, so it is exact in both
 * single and double precision, and the set of values is symmetric about 1/2. */
static double u01(uint32_t w) { return ((double)(w >> 9) + 0.5) * (1.0 / 8388608.0); }

ORACLE_API double oracle_u01(uint32_t w) { return u01(w); }

/* ------------------------------------------------------------------------ */
/* Parameters, geometry.                                                    */
/* ------------------------------------------------------------------------ */
enum { J_UNIFORM = 0, J_PM = 1, J_FP32 = 2 };

typedef struct {
  int32_t d, n, L;
  int32_t J_kind;       /* J_UNIFORM: J_ij = J0; J_PM: J0 * (+-1) int8; J_FP32 */
  uint64_t seed;
  uint32_t replica;
  int32_t renorm_every; /* continuous spins: renormalise after sweeps t % R == 0 */
  double J0;
  double J_sigma;       /* Gaussian couplings: J = J0 + sigma * N(0,1) */
  double delta;         /* XY: max rotation angle; Heisenberg: cap half-angle */
} oracle_params;

typedef struct {
  int64_t n_attempt;
  int64_t n_accept;
  int64_t dE_units;     /* Ising with integer couplings: sum of accepted m (dE = 2 J0 m) */
  double dE;            /* sum of accepted energy changes, double */
  int64_t n_near;       /* continuous / FP32-J: |u - p| < 1e-6 */
} oracle_stats;

typedef struct {
  int64_t E_int;        /* -sum J_sign s_i s_j (Ising with uniform or +-1 couplings) */
  int64_t M_int;        /* sum s_i (Ising) */
  double E;             /* energy in units of J0 applied (double) */
  double M[3];          /* magnetisation vector */
  double absM;          /* |M| */
} oracle_obs;

static int64_t n_sites(const oracle_params *p) {
  int64_t N = 1;
  for (int k = 0; k < p->d; ++k) N *= p->L;
  return N;
}

static void coords(const oracle_params *p, int64_t i, int64_t x[3]) {
  int64_t L = p->L;
  x[0] = i % L;
  x[1] = (i / L) % L;
  x[2] = (p->d == 3) ? i / (L * L) : 0;
}

static int64_t site(const oracle_params *p, const int64_t x[3]) {
  int64_t L = p->L;
  return x[0] + L * x[1] + (p->d == 3 ? L * L * x[2] : 0);
}

static int colour_of(const oracle_params *p, int64_t i) {
  int64_t x[3];
  coords(p, i, x);
  return (int)((x[0] + x[1] + x[2]) & 1);
}

/* neighbour of i one step along axis mu in direction dir (+1 or -1), periodic */
static int64_t neighbour(const oracle_params *p, int64_t i, int mu, int dir) {
  int64_t x[3];
  coords(p, i, x);
  x[mu] = (x[mu] + dir + p->L) % p->L;
  return site(p, x);
}

static int valid(const oracle_params *p) {
  if (p->d != 2 && p->d != 3) return 0;
  if (p->n < 1 || p->n > 3) return 0;
  if (p->L < 2 || (p->L & 1)) return 0;
  if (p->J_kind < 0 || p->J_kind > 2) return 0;
  return 1;
}

/* coupling of the bond (i, i + mu) */
static double coupling(const oracle_params *p, const void *J, int mu, int64_t i) {
  int64_t N = n_sites(p);
  switch (p->J_kind) {
    case J_PM: return p->J0 * (double)((const int8_t *)J)[mu * N + i];
    case J_FP32: return (double)((const float *)J)[mu * N + i];
    default: return p->J0;
  }
}

/* integer sign of the bond coupling (uniform and +-J kinds) */
static int coupling_sign(const oracle_params *p, const void *J, int mu, int64_t i) {
  if (p->J_kind == J_PM) return ((const int8_t *)J)[mu * n_sites(p) + i];
  return 1;
}

/* ------------------------------------------------------------------------ */
/* Boltzmann thresholds (Sec. 2: pre-tabulated Boltzmann factors).          */
/* For dE > 0 the move is accepted iff u < exp(-beta dE) with u = u32/2^32, */
/* i.e. iff u32 < T(dE) = ceil(2^32 exp(-beta dE)).  Computed in long       */
/* double (64-bit significand).  dE <= 0 is always accepted; T = 2^32 also  */
/* means "always".                                                          */
/* ------------------------------------------------------------------------ */
ORACLE_API uint64_t oracle_threshold(double beta, double dE) {
  if (!(dE > 0.0)) return 4294967296ull;
  long double b = (long double)beta, e = (long double)dE;
  if (isinf(beta)) return 0;
  long double x = ldexpl(expl(-b * e), 32);
  long double c = ceill(x);
  if (c >= 4294967296.0L) return 4294967296ull;
  return (uint64_t)c;
}

/* ------------------------------------------------------------------------ */
/* Initialisation.                                                          */
/* ------------------------------------------------------------------------ */
ORACLE_API int oracle_init_ising(const oracle_params *p, int hot, int8_t *s) {
  if (!valid(p) || p->n != 1) return -1;
  int64_t N = n_sites(p);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    if (!hot) { s[i] = 1; continue; }
    uint32_t w[4];
    draw(p->seed, (uint32_t)(i >> 7), 0u, p->replica, (uint32_t)(PURPOSE_INIT_SPIN << 1), w);
    uint32_t bit = (w[(i >> 5) & 3] >> (i & 31)) & 1u;
    s[i] = bit ? (int8_t)-1 : (int8_t)1;
  }
  return 0;
}

/* continuous spins, components stored [n][N]; values rounded to single
 * precision (the GPU stores FP32 spins) and held as doubles */
ORACLE_API int oracle_init_continuous(const oracle_params *p, int hot, double *s) {
  if (!valid(p) || p->n < 2) return -1;
  int64_t N = n_sites(p);
  const double two_pi = 6.283185307179586476925286766559;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    double v[3] = {1.0, 0.0, 0.0};
    if (hot) {
      uint32_t w[4];
      draw(p->seed, (uint32_t)i, 0u, p->replica, (uint32_t)(PURPOSE_INIT_SPIN << 1), w);
      if (p->n == 2) {
        double th = two_pi * u01(w[0]);
        v[0] = cos(th); v[1] = sin(th);
      } else {
        double z = 2.0 * u01(w[0]) - 1.0, ph = two_pi * u01(w[1]);
        double r = sqrt(1.0 - z * z);
        v[0] = r * cos(ph); v[1] = r * sin(ph); v[2] = z;
      }
    }
    for (int k = 0; k < p->n; ++k) s[k * N + i] = (double)(float)v[k];
  }
  return 0;
}

/* couplings [d][N]: int8 +-1 for J_PM, float for J_FP32 (Gaussian) */
ORACLE_API int oracle_init_couplings(const oracle_params *p, void *J) {
  if (!valid(p)) return -1;
  int64_t N = n_sites(p);
  const double two_pi = 6.283185307179586476925286766559;
  if (p->J_kind != J_PM && p->J_kind != J_FP32) return -1;
  for (int mu = 0; mu < p->d; ++mu) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
      uint32_t w[4];
      if (p->J_kind == J_PM) {
        draw(p->seed, (uint32_t)(i >> 7), (uint32_t)mu, p->replica,
             (uint32_t)(PURPOSE_COUPLING << 1), w);
        uint32_t bit = (w[(i >> 5) & 3] >> (i & 31)) & 1u;
        ((int8_t *)J)[mu * N + i] = bit ? (int8_t)-1 : (int8_t)1;
      } else if (p->J_kind == J_FP32) {
        draw(p->seed, (uint32_t)i, (uint32_t)mu, p->replica, (uint32_t)(PURPOSE_COUPLING << 1), w);
        double g = sqrt(-2.0 * log(u01(w[0]))) * cos(two_pi * u01(w[1]));
        ((float *)J)[mu * N + i] = (float)(p->J0 + p->J_sigma * g);
      }
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Local field h_i = sum_mu [J(i,mu) s_{i+mu} + J(i-mu,mu) s_{i-mu}],       */
/* accumulated in the order +x, -x, +y, -y, +z, -z.                          */
/* ------------------------------------------------------------------------ */
static void local_field(const oracle_params *p, const double *s, const void *J, int64_t i,
                        double h[3]) {
  int64_t N = n_sites(p);
  h[0] = h[1] = h[2] = 0.0;
  for (int mu = 0; mu < p->d; ++mu) {
    int64_t ip = neighbour(p, i, mu, +1), im = neighbour(p, i, mu, -1);
    double jp = coupling(p, J, mu, i), jm = coupling(p, J, mu, im);
    for (int k = 0; k < p->n; ++k) h[k] += jp * s[k * N + ip];
    for (int k = 0; k < p->n; ++k) h[k] += jm * s[k * N + im];
  }
}

/* ------------------------------------------------------------------------ */
/* One half-sweep: every site of colour c attempts one Metropolis move      */
/* against the current configuration of the other colour (Sec. 2).  Sites of */
/* one colour have no bonds among themselves, so updating them in place in  */
/* any order gives the same result as updating them simultaneously.         */
/* margin (optional, natural order, length N): u - p for sites whose        */
/* decision involved a floating-point probability, NAN otherwise.           */
/* ------------------------------------------------------------------------ */
static uint32_t site_index_in_colour(int64_t i) { return (uint32_t)(i >> 1); }

/* Decision for Ising site i of colour c whose 2d neighbours (order +x, -x, +y,
 * -y, +z, -z) hold the spins nb[].  With integer couplings the move is
 * described by m_i = s_i * sum_b sign(J_b) s_b, dE = 2 J0 m_i.  T: thresholds per m in [-2d, 2d] (integer
 * couplings).  Returns 1 to flip.  m_out / dE_out / margin (optional) report
 * the move. */
static int ising_decide(const oracle_params *p, const void *J, double beta, const uint64_t *T,
                        uint32_t t, int c, int64_t i, int si, const int nb[6], int *m_out,
                        double *dE_out, double *margin) {
  int d = p->d;
  uint32_t j = site_index_in_colour(i);
  if (p->J_kind == J_FP32) {
    double h = 0.0;
    for (int mu = 0; mu < d; ++mu) {
      int64_t im = neighbour(p, i, mu, -1);
      h += coupling(p, J, mu, i) * (double)nb[2 * mu];
      h += coupling(p, J, mu, im) * (double)nb[2 * mu + 1];
    }
    double dE = 2.0 * (double)si * h;
    uint32_t w[4];
    draw(p->seed, j >> 2, t, p->replica, (uint32_t)(c | (PURPOSE_CONTINUOUS << 1)), w);
    double u = u01(w[j & 3]);
    if (dE_out) *dE_out = dE;
    if (m_out) *m_out = 0;
    if (dE <= 0.0) {
      if (margin) *margin = NAN;
      return 1;
    }
    double pr = exp(-beta * dE);
    if (margin) *margin = u - pr;
    return u < pr;
  }
  int sum = 0;
  for (int mu = 0; mu < d; ++mu) {
    int64_t im = neighbour(p, i, mu, -1);
    sum += coupling_sign(p, J, mu, i) * nb[2 * mu];
    sum += coupling_sign(p, J, mu, im) * nb[2 * mu + 1];
  }
  int m = si * sum;
  uint32_t wp[4], wr[4];
  draw(p->seed, j >> 4, t, p->replica, (uint32_t)(c | (PURPOSE_ISING_PREFIX << 1)), wp);
  draw(p->seed, j, t, p->replica, (uint32_t)(c | (PURPOSE_ISING_REFINE << 1)), wr);
  uint32_t prefix = (wp[(j >> 2) & 3] >> (8 * (j & 3))) & 0xffu;
  uint64_t u32 = ((uint64_t)prefix << 24) | (wr[0] & 0xffffffu);
  if (m_out) *m_out = m;
  if (dE_out) *dE_out = 2.0 * p->J0 * m;
  if (margin) *margin = NAN;
  return u32 < T[m + 2 * d];
}

static void gather_ising(const oracle_params *p, const int8_t *s, int64_t i, int nb[6]) {
  for (int mu = 0; mu < p->d; ++mu) {
    nb[2 * mu] = s[neighbour(p, i, mu, +1)];
    nb[2 * mu + 1] = s[neighbour(p, i, mu, -1)];
  }
}

static void ising_table(const oracle_params *p, double beta, uint64_t T[13]) {
  int d = p->d;
  for (int m = -2 * d; m <= 2 * d; ++m) T[m + 2 * d] = oracle_threshold(beta, 2.0 * p->J0 * m);
}

static int half_sweep_ising(const oracle_params *p, int8_t *s, const void *J, double beta,
                            uint32_t t, int c, oracle_stats *st, double *margin) {
  int64_t N = n_sites(p);
  uint64_t T[13];
  ising_table(p, beta, T);
  int64_t n_att = 0, n_acc = 0, dEu = 0, n_near = 0;
  double dEsum = 0.0;
#pragma omp parallel for schedule(static) if (N >= 65536) reduction(+ : n_att, n_acc, dEu, n_near, dEsum)
  for (int64_t i = 0; i < N; ++i) {
    if (colour_of(p, i) != c) continue;
    n_att++;
    int nb[6], m;
    double dE, mg;
    gather_ising(p, s, i, nb);
    int accept = ising_decide(p, J, beta, T, t, c, i, s[i], nb, &m, &dE, &mg);
    if (margin) margin[i] = mg;
    if (!isnan(mg) && fabs(mg) < 1e-6) n_near++;
    if (accept) {
      s[i] = (int8_t)-s[i];
      n_acc++;
      dEu += m;
      dEsum += dE;
    }
  }
  if (st) {
    st->n_attempt += n_att; st->n_accept += n_acc; st->dE_units += dEu;
    st->dE += dEsum; st->n_near += n_near;
  }
  return 0;
}

/* Spins of selected sites after one full sweep with counter t, computed from
 * the state s before the sweep (which is not modified): a colour-0 site needs
 * only its own update; a colour-1 site is updated against the colour-0
 * neighbours as the first half-sweep leaves them. */
ORACLE_API int oracle_ising_sweep_sites(const oracle_params *p, const int8_t *s, const void *J,
                                        double beta, uint64_t t, int64_t n_sel,
                                        const int64_t *sites, int8_t *out) {
  if (!valid(p) || p->n != 1 || t > 0xffffffffull) return -1;
  uint64_t T[13];
  ising_table(p, beta, T);
  int64_t N = n_sites(p);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n_sel; ++k) {
    int64_t i = sites[k];
    if (i < 0 || i >= N) { out[k] = 0; continue; }
    int nb[6];
    if (colour_of(p, i) == 0) {
      gather_ising(p, s, i, nb);
      int acc = ising_decide(p, J, beta, T, (uint32_t)t, 0, i, s[i], nb, NULL, NULL, NULL);
      out[k] = acc ? (int8_t)-s[i] : s[i];
      continue;
    }
    for (int mu = 0; mu < p->d; ++mu) {
      for (int dir = 0; dir < 2; ++dir) {
        int64_t q = neighbour(p, i, mu, dir == 0 ? +1 : -1);
        int nq[6];
        gather_ising(p, s, q, nq);
        int acc = ising_decide(p, J, beta, T, (uint32_t)t, 0, q, s[q], nq, NULL, NULL, NULL);
        nb[2 * mu + dir] = acc ? -s[q] : s[q];
      }
    }
    int acc = ising_decide(p, J, beta, T, (uint32_t)t, 1, i, s[i], nb, NULL, NULL, NULL);
    out[k] = acc ? (int8_t)-s[i] : s[i];
  }
  return 0;
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Proposal for a continuous spin (n = 2 rotation by Delta in [-delta, delta];
 * n = 3 uniform point on the spherical cap of half-angle delta around s). */
static void propose(const oracle_params *p, const double s[3], const uint32_t *wprop, double out[3]) {
  const double two_pi = 6.283185307179586476925286766559;
  if (p->n == 2) {
    double D = p->delta * (2.0 * u01(wprop[0]) - 1.0);
    double cD = cos(D), sD = sin(D);
    out[0] = s[0] * cD - s[1] * sD;
    out[1] = s[1] * cD + s[0] * sD;
    out[2] = 0.0;
    return;
  }
  double one_minus_cmax = 1.0 - cos(p->delta);
  double ca = 1.0 - u01(wprop[0]) * one_minus_cmax;
  double sa = sqrt(fmax(0.0, 1.0 - ca * ca));
  double ph = two_pi * u01(wprop[1]);
  /* frame: axis e_k with the smallest |s_k| (lowest k on ties) */
  int k = 0;
  for (int q = 1; q < 3; ++q)
    if (fabs(s[q]) < fabs(s[k])) k = q;
  double e1[3] = {0.0, 0.0, 0.0};
  e1[k] = 1.0;
  double sk = s[k];
  for (int q = 0; q < 3; ++q) e1[q] -= sk * s[q];
  double nrm = sqrt(dot3(e1, e1));
  for (int q = 0; q < 3; ++q) e1[q] /= nrm;
  double e2[3] = {s[1] * e1[2] - s[2] * e1[1], s[2] * e1[0] - s[0] * e1[2],
                  s[0] * e1[1] - s[1] * e1[0]};
  double cph = cos(ph), sph = sin(ph);
  for (int q = 0; q < 3; ++q) out[q] = ca * s[q] + sa * (cph * e1[q] + sph * e2[q]);
}

static int half_sweep_continuous(const oracle_params *p, double *s, const void *J, double beta,
                                 uint32_t t, int c, oracle_stats *st, double *margin) {
  int64_t N = n_sites(p);
  int n = p->n;
  int64_t n_att = 0, n_acc = 0, n_near = 0;
  double dEsum = 0.0;
  /* All colour-c sites see only colour-(1-c) neighbours, so the proposals can
   * be applied in place. */
#pragma omp parallel for schedule(static) if (N >= 65536) reduction(+ : n_att, n_acc, n_near, dEsum)
  for (int64_t i = 0; i < N; ++i) {
    if (colour_of(p, i) != c) continue;
    uint32_t j = site_index_in_colour(i);
    n_att++;
    double h[3], si[3] = {0.0, 0.0, 0.0}, sn[3];
    local_field(p, s, J, i, h);
    for (int k = 0; k < n; ++k) si[k] = s[k * N + i];
    uint32_t w[4];
    uint32_t wacc, wprop[2];
    if (n == 2) {
      draw(p->seed, j >> 1, t, p->replica, (uint32_t)(c | (PURPOSE_CONTINUOUS << 1)), w);
      wacc = w[2 * (j & 1)];
      wprop[0] = w[2 * (j & 1) + 1];
      wprop[1] = 0;
    } else {
      draw(p->seed, j, t, p->replica, (uint32_t)(c | (PURPOSE_CONTINUOUS << 1)), w);
      wacc = w[0];
      wprop[0] = w[1];
      wprop[1] = w[2];
    }
    propose(p, si, wprop, sn);
    double dE = 0.0;
    for (int k = 0; k < n; ++k) dE -= (sn[k] - si[k]) * h[k];
    int accept;
    if (dE <= 0.0) {
      accept = 1;
      if (margin) margin[i] = NAN;
    } else {
      double u = u01(wacc), pr = exp(-beta * dE);
      accept = u < pr;
      if (margin) margin[i] = u - pr;
      if (fabs(u - pr) < 1e-6) n_near++;
    }
    if (accept) {
      for (int k = 0; k < n; ++k) s[k * N + i] = sn[k];
      n_acc++;
      dEsum += dE;
    }
  }
  if (st) {
    st->n_attempt += n_att; st->n_accept += n_acc; st->dE += dEsum; st->n_near += n_near;
  }
  return 0;
}

ORACLE_API int oracle_half_sweep(const oracle_params *p, void *s, const void *J, double beta,
                                 uint64_t t, int c, oracle_stats *st, double *margin) {
  if (!valid(p) || (c != 0 && c != 1) || t > 0xffffffffull) return -1;
  if (!(beta >= 0.0)) return -1;
  if (p->J_kind != J_UNIFORM && J == NULL) return -1;
  if (p->n == 1) return half_sweep_ising(p, (int8_t *)s, J, beta, (uint32_t)t, c, st, margin);
  return half_sweep_continuous(p, (double *)s, J, beta, (uint32_t)t, c, st, margin);
}

ORACLE_API void oracle_renormalize(const oracle_params *p, double *s) {
  int64_t N = n_sites(p);
  for (int64_t i = 0; i < N; ++i) {
    double q = 0.0;
    for (int k = 0; k < p->n; ++k) q += s[k * N + i] * s[k * N + i];
    double r = sqrt(q);
    for (int k = 0; k < p->n; ++k) s[k * N + i] /= r;
  }
}

/* ------------------------------------------------------------------------ */
/* Observables: E = -sum_i sum_mu J(i,mu) s_i . s_{i+mu} (each bond once),   */
/* M = sum_i s_i.  Integer sums for Ising with integer couplings.           */
/* ------------------------------------------------------------------------ */
ORACLE_API void oracle_measure(const oracle_params *p, const void *s, const void *J,
                               oracle_obs *out) {
  int64_t N = n_sites(p);
  memset(out, 0, sizeof(*out));
  if (p->n == 1) {
    const int8_t *si = (const int8_t *)s;
    int64_t Ei = 0, Mi = 0;
    double Ef = 0.0;
#pragma omp parallel for schedule(static) if (N >= 65536) reduction(+ : Ei, Mi, Ef)
    for (int64_t i = 0; i < N; ++i) {
      Mi += si[i];
      for (int mu = 0; mu < p->d; ++mu) {
        int64_t ip = neighbour(p, i, mu, +1);
        if (p->J_kind == J_FP32)
          Ef -= coupling(p, J, mu, i) * (double)(si[i] * si[ip]);
        else
          Ei -= (int64_t)coupling_sign(p, J, mu, i) * si[i] * si[ip];
      }
    }
    out->E_int = Ei;
    out->M_int = Mi;
    out->E = (p->J_kind == J_FP32) ? Ef : p->J0 * (double)Ei;
    out->M[0] = (double)Mi;
    out->absM = fabs((double)Mi);
    return;
  }
  const double *sv = (const double *)s;
  double E = 0.0, M0 = 0.0, M1 = 0.0, M2 = 0.0;
#pragma omp parallel for schedule(static) if (N >= 65536) reduction(+ : E, M0, M1, M2)
  for (int64_t i = 0; i < N; ++i) {
    M0 += sv[i];
    M1 += sv[N + i];
    if (p->n == 3) M2 += sv[2 * N + i];
    for (int mu = 0; mu < p->d; ++mu) {
      int64_t ip = neighbour(p, i, mu, +1);
      double dp = 0.0;
      for (int k = 0; k < p->n; ++k) dp += sv[k * N + i] * sv[k * N + ip];
      E -= coupling(p, J, mu, i) * dp;
    }
  }
  out->E = E;
  out->M[0] = M0; out->M[1] = M1; out->M[2] = M2;
  out->absM = sqrt(M0 * M0 + M1 * M1 + M2 * M2);
}

/* Bond correlations: acc[mu][i] += s_i . s_{i+mu}.  int64 for Ising, double
 * for continuous spins. */
ORACLE_API void oracle_bond_accumulate(const oracle_params *p, const void *s, void *acc) {
  int64_t N = n_sites(p);
  for (int mu = 0; mu < p->d; ++mu) {
#pragma omp parallel for schedule(static) if (N >= 65536)
    for (int64_t i = 0; i < N; ++i) {
      int64_t ip = neighbour(p, i, mu, +1);
      if (p->n == 1) {
        const int8_t *si = (const int8_t *)s;
        ((int64_t *)acc)[mu * N + i] += (int64_t)(si[i] * si[ip]);
      } else {
        const double *sv = (const double *)s;
        double dp = 0.0;
        for (int k = 0; k < p->n; ++k) dp += sv[k * N + i] * sv[k * N + ip];
        ((double *)acc)[mu * N + i] += dp;
      }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Sweeps: for each t, colour 0 then colour 1, then t += 1; continuous      */
/* spins are renormalised after sweeps with t % renorm_every == 0.  Every   */
/* measure_every sweeps (if > 0) the observables are appended to series.    */
/* ------------------------------------------------------------------------ */
ORACLE_API int oracle_sweeps(const oracle_params *p, void *s, const void *J, double beta,
                             uint64_t t0, int64_t n_sweeps, int64_t measure_every,
                             oracle_obs *series, oracle_stats *st) {
  if (!valid(p) || n_sweeps < 0) return -1;
  if (t0 + (uint64_t)n_sweeps > 0x100000000ull) return -1;
  int64_t k = 0;
  for (int64_t q = 0; q < n_sweeps; ++q) {
    uint64_t t = t0 + (uint64_t)q;
    for (int c = 0; c < 2; ++c) {
      int rc = oracle_half_sweep(p, s, J, beta, t, c, st, NULL);
      if (rc) return rc;
    }
    uint64_t tn = t + 1;
    if (p->n > 1 && p->renorm_every > 0 && tn % (uint64_t)p->renorm_every == 0)
      oracle_renormalize(p, (double *)s);
    if (measure_every > 0 && (q + 1) % measure_every == 0 && series)
      oracle_measure(p, s, J, &series[k++]);
  }
  return 0;
}

/* Many independent chains of a small lattice from one starting state:
 * replica r = replica0 + k for k < n_chains; states out [n_chains][N]. */
ORACLE_API int oracle_ensemble_ising(const oracle_params *p, const int8_t *s0, const void *J,
                                     double beta, uint64_t t0, int64_t n_sweeps,
                                     int64_t n_chains, int8_t *out) {
  if (!valid(p) || p->n != 1) return -1;
  int64_t N = n_sites(p);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t k = 0; k < n_chains; ++k) {
    oracle_params q = *p;
    q.replica = p->replica + (uint32_t)k;
    int8_t *s = out + k * N;
    memcpy(s, s0, (size_t)N);
    for (int64_t w = 0; w < n_sweeps; ++w) {
      half_sweep_ising(&q, s, J, beta, (uint32_t)(t0 + (uint64_t)w), 0, NULL, NULL);
      half_sweep_ising(&q, s, J, beta, (uint32_t)(t0 + (uint64_t)w), 1, NULL, NULL);
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Update rules and the tiled k-hit schedule (Sec. 2).                      */
/*                                                                          */
/* Heat bath: the new spin is +1 with probability                           */
/*   p_+ = 1 / (1 + exp(-2 beta h)),  h = J0 sum_nb sign(J) s_nb,          */
/* whatever the old spin; with u = u32 / 2^32 (the Metropolis draw: prefix  */
/* byte and 24-bit refinement), s = +1 iff u32 < T_hb = ceil(2^32 p_+).     */
/*                                                                          */
/* Tiled k-hit schedule: the lattice is cut into tiles of edge T (L/T even),*/
/* tiles coloured by (tx + ty + tz) mod 2.  A sweep treats tile colour 0,   */
/* then tile colour 1; for one tile colour, k times: every site of colour 0 */
/* in those tiles, then every site of colour 1 (the neighbouring tiles stay */
/* fixed meanwhile).  Every site is attempted k times per sweep.  Hit h of  */
/* sweep t uses counter word 3 = colour | purpose << 1 | h << 8 (h = 0 is   */
/* the plain sweep's counter).                                              */
/* ------------------------------------------------------------------------ */
ORACLE_API uint64_t oracle_threshold_hb(double beta, double h) {
  if (isinf(beta)) return h > 0.0 ? 4294967296ull : (h < 0.0 ? 0ull : 2147483648ull);
  long double b = (long double)beta, e = (long double)h;
  long double x = ldexpl(1.0L / (1.0L + expl(-2.0L * b * e)), 32);
  long double c = ceill(x);
  if (c >= 4294967296.0L) return 4294967296ull;
  return (uint64_t)c;
}

static int tile_colour(const oracle_params *p, int64_t i, int T) {
  int64_t x[3];
  coords(p, i, x);
  return (int)((x[0] / T + x[1] / T + (p->d == 3 ? x[2] / T : 0)) & 1);
}

/* New spin of Ising site i (integer couplings) under rule 0 (Metropolis) or
 * 1 (heat bath), with counter (block, t, replica, c | purpose<<1 | hit<<8). */
static int ising_rule_site(const oracle_params *p, const int8_t *s, const void *J,
                           const uint64_t *Tm, const uint64_t *Th, uint32_t t, int c,
                           uint32_t hit, int rule, int64_t i) {
  int d = p->d;
  uint32_t j = site_index_in_colour(i);
  int sum = 0;  /* sum_nb sign(J) s_nb */
  for (int mu = 0; mu < d; ++mu) {
    int64_t ip = neighbour(p, i, mu, +1), im = neighbour(p, i, mu, -1);
    sum += coupling_sign(p, J, mu, i) * s[ip];
    sum += coupling_sign(p, J, mu, im) * s[im];
  }
  uint32_t wp[4], wr[4];
  draw(p->seed, j >> 4, t, p->replica, (uint32_t)c | (PURPOSE_ISING_PREFIX << 1) | (hit << 8), wp);
  draw(p->seed, j, t, p->replica, (uint32_t)c | (PURPOSE_ISING_REFINE << 1) | (hit << 8), wr);
  uint32_t prefix = (wp[(j >> 2) & 3] >> (8 * (j & 3))) & 0xffu;
  uint64_t u32 = ((uint64_t)prefix << 24) | (wr[0] & 0xffffffu);
  if (rule == 1) return u32 < Th[sum + 2 * d] ? 1 : -1;
  int m = s[i] * sum;  /* dE = 2 J0 m */
  return u32 < Tm[m + 2 * d] ? -s[i] : s[i];
}

/* Thresholds of both rules for dE = 2 J0 m (Metropolis) and h = J0 m (heat
 * bath), m = -2d..2d. */
static void rule_tables(const oracle_params *p, double beta, uint64_t Tm[13], uint64_t Th[13]) {
  int d = p->d;
  for (int m = -2 * d; m <= 2 * d; ++m) {
    Tm[m + 2 * d] = oracle_threshold(beta, 2.0 * p->J0 * m);
    Th[m + 2 * d] = oracle_threshold_hb(beta, p->J0 * m);
  }
}

/* One pass over tile colour tc (tile > 0) or over the whole lattice (tile =
 * 0): `hits` times, every selected site of colour 0 and then every selected
 * site of colour 1 attempts one move against the state the previous stage
 * left; all other sites stay fixed.  nw: scratch of N bytes. */
static void rule_pass(const oracle_params *p, int8_t *s, const void *J, const uint64_t *Tm,
                      const uint64_t *Th, uint32_t t, int rule, int tile, int tc, int hits,
                      int8_t *nw) {
  int64_t N = n_sites(p);
  for (int h = 0; h < hits; ++h)
    for (int c = 0; c < 2; ++c) {
      /* all selected sites at once from the same state (they are independent) */
#pragma omp parallel for schedule(static) if (N >= 65536)
      for (int64_t i = 0; i < N; ++i) {
        int sel = colour_of(p, i) == c && (tile == 0 || tile_colour(p, i, tile) == tc);
        nw[i] = sel ? (int8_t)ising_rule_site(p, s, J, Tm, Th, t, c, (uint32_t)h, rule, i) : s[i];
      }
      memcpy(s, nw, (size_t)N);
    }
}

static int rule_args_ok(const oracle_params *p, int rule, int tile, int hits) {
  if (!valid(p) || p->n != 1 || p->J_kind == J_FP32 || (rule != 0 && rule != 1)) return 0;
  if (tile < 0 || (tile > 0 && (p->L % tile || ((p->L / tile) & 1) || hits < 1 || hits > (1 << 23))))
    return 0;
  return 1;
}

/* n_sweeps sweeps of an Ising lattice with integer couplings under `rule`,
 * plain (tile = 0: colour 0 then colour 1, hit 0) or tiled k-hit (tile T,
 * hits k >= 1: the pass over tile colour 0, then the pass over tile colour
 * 1).  The counter of sweep q is t0 + q. */
ORACLE_API int oracle_sweeps_rule(const oracle_params *p, int8_t *s, const void *J, double beta,
                                  uint64_t t0, int64_t n_sweeps, int rule, int tile, int hits) {
  if (!rule_args_ok(p, rule, tile, hits)) return -1;
  if (n_sweeps < 0 || t0 + (uint64_t)n_sweeps > 0x100000000ull) return -1;
  uint64_t Tm[13], Th[13];
  rule_tables(p, beta, Tm, Th);
  int8_t *nw = (int8_t *)malloc((size_t)n_sites(p));
  if (!nw) return -2;
  int passes = tile > 0 ? 2 : 1, k = tile > 0 ? hits : 1;
  for (int64_t q = 0; q < n_sweeps; ++q) {
    uint32_t t = (uint32_t)(t0 + (uint64_t)q);
    for (int tc = 0; tc < passes; ++tc) rule_pass(p, s, J, Tm, Th, t, rule, tile, tc, k, nw);
  }
  free(nw);
  return 0;
}

/* The pass over tile colour tc alone (tile > 0), with counter t: one half of
 * a tiled sweep. */
ORACLE_API int oracle_tile_pass(const oracle_params *p, int8_t *s, const void *J, double beta,
                                uint64_t t, int rule, int tile, int hits, int tc) {
  if (!rule_args_ok(p, rule, tile, hits) || tile == 0 || (tc != 0 && tc != 1)) return -1;
  if (t > 0xffffffffull) return -1;
  uint64_t Tm[13], Th[13];
  rule_tables(p, beta, Tm, Th);
  int8_t *nw = (int8_t *)malloc((size_t)n_sites(p));
  if (!nw) return -2;
  rule_pass(p, s, J, Tm, Th, (uint32_t)t, rule, tile, tc, hits, nw);
  free(nw);
  return 0;
}

/* Chains for derivatives of ln Z (Eq. (1)): n_chains independent chains of
 * one small lattice, chain k with replica p->replica + k, its own start state
 * s0[k] and the shared couplings J.  After every sweep the bond products
 * s_i s_{i+mu} of every chain are added to bond_sum[mu][i] (natural order)
 * and, if samples is not NULL, stored in samples[k][w][mu][i].  min_margin
 * receives the smallest |u - exp(-beta dE)| over all uphill decisions (how
 * close an FP32 implementation could come to deciding differently); it is
 * +inf when no decision used a threshold. */
ORACLE_API int oracle_chains_ising(const oracle_params *p, const int8_t *s0, const void *J,
                                   double beta, uint64_t t0, int64_t n_sweeps, int64_t n_chains,
                                   int8_t *out, int64_t *bond_sum, int8_t *samples,
                                   double *min_margin) {
  if (!valid(p) || p->n != 1 || n_sweeps < 0 || n_chains < 1) return -1;
  if (t0 + (uint64_t)n_sweeps > 0x100000000ull) return -1;
  int64_t N = n_sites(p);
  int d = p->d;
  int64_t *part = (int64_t *)calloc((size_t)(n_chains * d * N), sizeof(int64_t));
  double *mins = (double *)malloc((size_t)n_chains * sizeof(double));
  if (!part || !mins) { free(part); free(mins); return -2; }
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t k = 0; k < n_chains; ++k) {
    oracle_params q = *p;
    q.replica = p->replica + (uint32_t)k;
    int8_t *s = out + k * N;
    memcpy(s, s0 + k * N, (size_t)N);
    double *mg = (double *)malloc((size_t)N * sizeof(double));
    double mn = INFINITY;
    for (int64_t w = 0; w < n_sweeps; ++w) {
      for (int c = 0; c < 2; ++c) {
        half_sweep_ising(&q, s, J, beta, (uint32_t)(t0 + (uint64_t)w), c, NULL, mg);
        for (int64_t i = 0; i < N; ++i)
          if (colour_of(p, i) == c && !isnan(mg[i]) && fabs(mg[i]) < mn) mn = fabs(mg[i]);
      }
      for (int mu = 0; mu < d; ++mu)
        for (int64_t i = 0; i < N; ++i) {
          int8_t v = (int8_t)(s[i] * s[neighbour(p, i, mu, +1)]);
          part[(k * d + mu) * N + i] += v;
          if (samples) samples[((k * n_sweeps + w) * d + mu) * N + i] = v;
        }
    }
    mins[k] = mn;
    free(mg);
  }
  double mn = INFINITY;
  for (int64_t k = 0; k < n_chains; ++k) {
    for (int64_t b = 0; b < d * N; ++b) bond_sum[b] += part[k * d * N + b];
    if (mins[k] < mn) mn = mins[k];
  }
  if (min_margin) *min_margin = mn;
  free(part);
  free(mins);
  return 0;
}

ORACLE_API int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the OpenMP loops (n <= 0: one per processor); for timing the
 * oracle on one core and on all of them. */
ORACLE_API void oracle_set_num_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
#else
  (void)n;
#endif
}
