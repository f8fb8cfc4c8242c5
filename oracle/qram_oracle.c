/*
 * qram_oracle.c -- plain CPU oracle for amplitude-damped bucket-brigade QRAM
 * trajectories (full, unpruned evolution of every branch).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the package's smoke check and the
 * benchmark's cpu_baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the HIP library: every quantity
 * below (random numbers, thresholds, schedule, gates, Kraus layers, fidelity)
 * is computed here from the paper's definitions, on its own.
 *
 * What it computes, per trajectory (paper: Sec. II A-B, Sec. IV D, App. A,
 * App. C):
 *   1. The damping candidate history: every (slice, tree site) pair is a
 *      candidate with probability gamma, drawn in advance and state
 *      independently (Sec. IV D, first step of the joint sampler).
 *   2. The brute-force bad-address set of the marking rule: Eq. (subtree)
 *      for the qutrit encoding, Eq. (badrange) for the qubit encoding.
 *   3. The full sparse evolution of the data-loading input
 *      sum_i c_i |i>|0>_bus|ground>_tree: each time slice applies its gates
 *      (bucket-brigade schedule with T = 6n+2k), then one joint damping layer
 *      over all M = 2(2^n-1) tree sites (Eq. layerkraus, Theorem 4):
 *      one auxiliary draw of a component x with probability |c_x|^2,
 *      J = C_s intersect X(x), then K_J applied to every component.
 *   4. The end of the query: the second Hadamard wall (qubit encoding), the
 *      tree measurement, and the fidelity of the post-measurement state with
 *      the ideal output sum_i c_i |i>|d_i>|ground> (Eq. nk-qram, App. C).
 *   Optionally (the _ex entry points): depolarizing faults of strength eps
 *   (Sec. II B; placement of App. C), drawn in advance like the damping
 *   candidates, applied as unitaries after the gates of their slice and
 *   before its damping layer, and marked by the same rule; and a general
 *   input sum_i c_i |i>|j_i> with one bus word per address (Sec. IV D).
 *
 * Conventions fixed here where the paper is silent (they are restated in the
 * design notes):
 *   - Address bit t (t = 0 .. n-1) is the bit routed at tree layer t, the
 *     most significant bit at the root: i_t = (i >> (n-1-t)) & 1.
 *   - Node v has children 2v+1 (left: router 0 / L) and 2v+2 (right: 1 / R).
 *     Site q = 2v is the router (qubit a_v, qutrit r_v), q = 2v+1 the data
 *     slot d_v.
 *   - Qutrit circuit: router qutrit {W,L,R} plus a data-slot qubit.  STORE on
 *     layer t acts on the node its parent routes into (the root for t = 0)
 *     and exchanges (W,b) <-> (L if b = 0 else R, 0).  A W router blocks the
 *     controlled swap.  FETCH is d_v ^= bit_b(m[2p + (r_v == R)]) when
 *     r_v != W.  No walls.
 *   - Random numbers: Philox4x32-10 keyed by the 64-bit seed; counters
 *     (block, draw, trajectory, 1) for candidates, (slice, 0, trajectory, 2)
 *     for the auxiliary draw of a damping layer, (0, 0, trajectory, 3) for the
 *     final tree measurement.  u64 = w0 | w1 << 32, u = (u64 >> 11) 2^-53.
 *   - The candidate set is sampled as i.i.d. Bernoulli(gamma) over the linear
 *     index L = (s-1) M + q by a geometric walk in 64-site blocks, whose gap
 *     thresholds are G[o] = floor(2^64 (1 - (1-gamma)^(o+1))) (saturated),
 *     with (1-gamma)^(o+1) formed by o+1 successive double multiplications.
 *   - Order of the auxiliary draw: all components whose mask C_s cap X(x) is
 *     empty come first as one block, then the remaining components in the
 *     order of their initial label (address, then bus word).  The same rule
 *     orders the final tree measurement: the ground-configuration block
 *     first.  Any fixed order samples the distribution of Theorem 4.
 *   - Amplitudes are kept unnormalised; draws use ratios (Sec. II B).
 *   - Depolarizing placement (pinned by the Pauli and Mixed rows of Table 4):
 *     in slice s the active positions are every site of the layers above the
 *     leaf layer whose router holds its address bit both before and after
 *     the gates of s (address bit t is stored at 3t+2 and unstored at
 *     T-3t-2), a prefix of the site numbering.  Each active position suffers
 *     a fault with probability eps; the faults form a geometric walk in
 *     64-site blocks over the linear index L = (active positions of slices
 *     1..s-1) + q, counters (block, draw, trajectory, 4).  The type comes from
 *     word w2 of the same draw: qubits (and the qutrit data slot) take X, Z
 *     or ZX = iY, index (w2 * 3) >> 32; a qutrit router takes one of the
 *     eight nontrivial Weyl operators, index (w2 * 8) >> 32 into (a, b) =
 *     (0,1) (0,2) (1,0) (1,1) (1,2) (2,0) (2,1) (2,2).  A fault (a, b) maps
 *     level x to x + a (mod d), then multiplies by w_d^(b (x + a)), w_2 = -1,
 *     w_3 = exp(2 pi i / 3); qubit X = (1,0), Z = (0,1), ZX = (1,1).
 *     Within a slice: gates, then the slice's depolarizing faults, then its
 *     damping layer.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_QUTRIT 0
#define ORC_QUBIT 1

#define ORC_TAG_FAULT 1u
#define ORC_TAG_AUX 2u
#define ORC_TAG_FINAL 3u
#define ORC_TAG_DEPOL 4u

/* qutrit router levels; a qubit site uses 0/1 */
#define LV_W 0
#define LV_L 1
#define LV_R 2

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11): ten rounds of the   */
/* Philox S-box on a 4x32-bit counter, key bumped by the Weyl constants     */
/* between rounds.                                                          */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)p1;
    uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)p0;
    x0 = y0;
    x1 = y1;
    x2 = y2;
    x3 = y3;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

static uint64_t draw_u64(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t traj,
                         uint32_t tag) {
  uint32_t ctr[4] = {c0, c1, traj, tag};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  return (uint64_t)w[0] | ((uint64_t)w[1] << 32);
}

static void draw_words(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t traj,
                       uint32_t tag, uint32_t w[4]) {
  uint32_t ctr[4] = {c0, c1, traj, tag};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  orc_philox4x32_10(ctr, key, w);
}

static double u53(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

double orc_uniform(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t traj,
                   uint32_t tag) {
  return u53(draw_u64(seed, c0, c1, traj, tag));
}

/* Gap thresholds of the geometric candidate walk. */
void orc_thresholds(double gamma, uint64_t G[64]) {
  double q = 1.0 - gamma;
  double qp = 1.0;
  for (int o = 0; o < 64; ++o) {
    qp = qp * q;
    double x = ldexp(1.0 - qp, 64);
    if (x >= 18446744073709551616.0)
      G[o] = UINT64_MAX;
    else
      G[o] = (uint64_t)x;
  }
}

/* ------------------------------------------------------------------------ */
/* Configuration and schedule (Sec. II A Eq. schedule; App. C).             */
/* ------------------------------------------------------------------------ */
enum { EV_COPY = 1, EV_STORE = 2, EV_CSWAP = 3, EV_BUS = 4, EV_FETCH = 5 };

#define ORC_MAXEV 64

typedef struct {
  int n, k, enc;
  int T, M, D, K2, E;
  double gamma, a, sg;
  const uint32_t *mem;
  uint64_t G[64];
  /* depolarizing faults and general inputs (zero / NULL: none, uniform) */
  double eps;
  uint64_t Gp[64];
  int nact[512];          /* active positions of slice s: sites 0 .. nact-1 */
  uint64_t dep_off[513];  /* linear index of slice s's first active position */
  double complex *cin;    /* normalised input amplitude of each address */
  uint32_t *jin;          /* input bus word of each address */
  double complex *cab;    /* or: normalised amplitude of each (address, bus
                             word) pair, 2^k per address */
  uint8_t *single;        /* cab: the address holds exactly one bus word */
  int wmax;               /* output words of the predicted good branches kept
                             up to this Hamming weight (-1: all) */
  int nev[512];
  int ev_type[512][ORC_MAXEV];
  int ev_arg[512][ORC_MAXEV];
} orc_cfg;

static void add_event(orc_cfg *c, int s, int type, int arg) {
  /* a layer's controlled swap fires once per slice, whoever lists it */
  for (int e = 0; e < c->nev[s]; ++e)
    if (c->ev_type[s][e] == type && c->ev_arg[s][e] == arg)
      return;
  c->ev_type[s][c->nev[s]] = type;
  c->ev_arg[s][c->nev[s]] = arg;
  c->nev[s]++;
}

/* Events of the bucket-brigade query.  Address bit t is copied into the root
 * data slot at 2t+1, moves down one layer per slice and is stored into the
 * router of layer t at 3t+2; data bit b enters at tau_in = 2n+2b+1, reaches
 * the leaf layer for the fetch at tau_fetch = 3n+2b+1 and leaves at
 * tau_out = 4n+2b+1 (Eq. schedule).  Every event at slice s has its mirror
 * at T-s. */
static void build_schedule(orc_cfg *c) {
  int n = c->n, k = c->k, T = c->T;
  memset(c->nev, 0, sizeof(c->nev));
  for (int t = 0; t < n; ++t) {
    add_event(c, 2 * t + 1, EV_COPY, t);
    add_event(c, T - 2 * t - 1, EV_COPY, t);
    for (int l = 0; l < t; ++l) {
      add_event(c, 2 * t + 2 + l, EV_CSWAP, l);
      add_event(c, T - 2 * t - 2 - l, EV_CSWAP, l);
    }
    add_event(c, 3 * t + 2, EV_STORE, t);
    add_event(c, T - 3 * t - 2, EV_STORE, t);
  }
  for (int b = 0; b < k; ++b) {
    add_event(c, 2 * n + 2 * b + 1, EV_BUS, b);
    add_event(c, 4 * n + 2 * b + 1, EV_BUS, b);
    for (int l = 0; l + 1 < n; ++l) {
      add_event(c, 2 * n + 2 * b + 2 + l, EV_CSWAP, l);
      add_event(c, 4 * n + 2 * b - l, EV_CSWAP, l);
    }
    add_event(c, 3 * n + 2 * b + 1, EV_FETCH, b);
  }
}

static int cfg_init(orc_cfg *c, int n, int k, int enc, double gamma,
                    const uint32_t *mem) {
  if (n < 1 || n > 15 || k < 1 || k > 8 || k > n)
    return -4;
  if (enc != ORC_QUBIT && enc != ORC_QUTRIT)
    return -1;
  if (!(gamma >= 0.0 && gamma < 1.0))
    return -1;
  c->n = n;
  c->k = k;
  c->enc = enc;
  c->T = 6 * n + 2 * k;
  c->M = 2 * ((1 << n) - 1);
  c->D = 1 << n;
  c->K2 = 1 << k;
  c->E = enc == ORC_QUBIT ? c->D * c->K2 : c->D;
  c->gamma = gamma;
  c->a = sqrt(1.0 - gamma);
  c->sg = sqrt(gamma);
  c->mem = mem;
  orc_thresholds(gamma, c->G);
  build_schedule(c);
  c->eps = 0.0;
  c->cin = NULL;
  c->jin = NULL;
  c->cab = NULL;
  c->single = NULL;
  c->wmax = -1;
  memset(c->nact, 0, sizeof(c->nact));
  memset(c->dep_off, 0, sizeof(c->dep_off));
  return 0;
}

/* Layers whose router holds its address bit both before and after the gates
 * of slice s, among the layers above the leaf layer (App. C placement). */
static int active_layers(const orc_cfg *c, int s) {
  int l = 0;
  for (int t = 0; t + 1 < c->n; ++t)
    if (3 * t + 2 < s && s < c->T - 3 * t - 2)
      ++l;
  return l;
}

/* Depolarizing strength and general input: cin (2 doubles per address) and
 * jin (bus word per address), or cab (2 doubles per (address, bus word),
 * address-major), or none (the data-loading input).  wmax >= 0 truncates
 * the predicted good branches' output words at that Hamming weight from
 * their ideal word (qubit encoding, one bus word per address).  Returns < 0
 * on bad input. */
static int cfg_extras(orc_cfg *c, double eps, const double *cin,
                      const uint32_t *jin, const double *cab, int wmax) {
  if (!(eps >= 0.0 && eps < 1.0))
    return -1;
  if (cab && (cin || jin))
    return -1;
  if (wmax < -1 || wmax > c->k)
    return -1;
  c->eps = eps;
  c->wmax = wmax == c->k ? -1 : wmax;
  orc_thresholds(eps, c->Gp);
  uint64_t off = 0;
  for (int s = 1; s < c->T; ++s) {
    int l = active_layers(c, s);
    c->nact[s] = 2 * ((1 << l) - 1);
    c->dep_off[s] = off;
    off += (uint64_t)c->nact[s];
  }
  c->dep_off[c->T] = off;
  if (cin) {
    double norm = 0.0;
    c->cin = (double complex *)malloc(sizeof(double complex) * c->D);
    for (int i = 0; i < c->D; ++i) {
      c->cin[i] = cin[2 * i] + I * cin[2 * i + 1];
      norm += creal(c->cin[i]) * creal(c->cin[i]) +
              cimag(c->cin[i]) * cimag(c->cin[i]);
    }
    if (!(norm > 0.0))
      return -1;
    for (int i = 0; i < c->D; ++i)
      c->cin[i] /= sqrt(norm);
  }
  if (jin) {
    c->jin = (uint32_t *)malloc(sizeof(uint32_t) * c->D);
    for (int i = 0; i < c->D; ++i)
      c->jin[i] = jin[i] & (uint32_t)(c->K2 - 1);
  }
  if (cab) {
    size_t na = (size_t)c->D * c->K2;
    double norm = 0.0;
    c->cab = (double complex *)malloc(sizeof(double complex) * na);
    c->single = (uint8_t *)malloc(c->D);
    for (size_t x = 0; x < na; ++x) {
      c->cab[x] = cab[2 * x] + I * cab[2 * x + 1];
      norm += cab[2 * x] * cab[2 * x] + cab[2 * x + 1] * cab[2 * x + 1];
    }
    if (!(norm > 0.0))
      return -1;
    for (size_t x = 0; x < na; ++x)
      c->cab[x] /= sqrt(norm);
    for (int i = 0; i < c->D; ++i) {
      int m = 0;
      for (int j = 0; j < c->K2; ++j)
        m += c->cab[(size_t)i * c->K2 + j] != 0.0;
      c->single[i] = m == 1;
      /* truncation is defined for one bus word per address (Theorem 2) */
      if (m > 1 && c->wmax >= 0)
        return -1;
    }
    /* the qutrit encoding carries one component per (address, bus word) */
    if (c->enc == ORC_QUTRIT)
      c->E = c->D * c->K2;
  }
  return 0;
}

static void cfg_free(orc_cfg *c) {
  if (!c)
    return;
  free(c->cin);
  free(c->jin);
  free(c->cab);
  free(c->single);
  free(c);
}

static double complex in_amp(const orc_cfg *c, uint32_t i) {
  return c->cin ? c->cin[i] : 1.0 / sqrt((double)c->D);
}

static uint32_t in_bus(const orc_cfg *c, uint32_t i) {
  return c->jin ? c->jin[i] : 0u;
}

/* Amplitude of (address i, bus word j) in the input. */
static double complex in_ab(const orc_cfg *c, uint32_t i, uint32_t j) {
  if (c->cab)
    return c->cab[(size_t)i * c->K2 + j];
  return j == in_bus(c, i) ? in_amp(c, i) : 0.0;
}

/* Does the input hold address i? */
static int present(const orc_cfg *c, uint32_t i) {
  if (!c->cab)
    return in_amp(c, i) != 0.0;
  for (int j = 0; j < c->K2; ++j)
    if (c->cab[(size_t)i * c->K2 + j] != 0.0)
      return 1;
  return 0;
}

/* The single bus word of address i (cab with one bus word, or cin/jin). */
static uint32_t single_bus(const orc_cfg *c, uint32_t i) {
  if (!c->cab)
    return in_bus(c, i);
  for (int j = 0; j < c->K2; ++j)
    if (c->cab[(size_t)i * c->K2 + j] != 0.0)
      return (uint32_t)j;
  return 0u;
}

/* Export the event list of slice s (for schedule tests). */
int orc_schedule(int n, int k, int s, int *types, int *args) {
  static const uint32_t zero_mem[1] = {0};
  orc_cfg *c = (orc_cfg *)calloc(1, sizeof(orc_cfg));
  int rc = cfg_init(c, n, k, ORC_QUBIT, 0.0, zero_mem);
  if (rc) {
    free(c);
    return rc;
  }
  int m = 0;
  if (s >= 1 && s < c->T) {
    m = c->nev[s];
    for (int e = 0; e < m; ++e) {
      types[e] = c->ev_type[s][e];
      args[e] = c->ev_arg[s][e];
    }
  }
  free(c);
  return m;
}

/* ------------------------------------------------------------------------ */
/* Candidate history (Sec. IV D step 1; Alg. 1 step 1).                      */
/* ------------------------------------------------------------------------ */
static int sample_candidates(const orc_cfg *c, uint64_t seed, uint32_t traj,
                             uint32_t *L, int cap) {
  uint64_t S = (uint64_t)(c->T - 1) * (uint64_t)c->M;
  uint64_t nb = (S + 63) / 64;
  int cnt = 0;
  for (uint64_t b = 0; b < nb; ++b) {
    uint64_t len = S - 64 * b < 64 ? S - 64 * b : 64;
    uint64_t pos = 0;
    for (uint32_t j = 0;; ++j) {
      uint64_t u = draw_u64(seed, (uint32_t)b, j, traj, ORC_TAG_FAULT);
      int o = 0;
      while (o < 64 && !(u < c->G[o]))
        ++o;
      if (o == 64 || pos + (uint64_t)o >= len)
        break;
      if (cnt < cap && L)
        L[cnt] = (uint32_t)(64 * b + pos + (uint64_t)o);
      ++cnt;
      pos += (uint64_t)o + 1;
    }
  }
  return cnt;
}

int orc_sample(int n, int k, double gamma, uint64_t seed, uint32_t traj,
               uint32_t *L, int cap) {
  static const uint32_t zero_mem[1] = {0};
  orc_cfg *c = (orc_cfg *)calloc(1, sizeof(orc_cfg));
  int rc = cfg_init(c, n, k, ORC_QUBIT, gamma, zero_mem);
  if (rc) {
    free(c);
    return rc;
  }
  int cnt = sample_candidates(c, seed, traj, L, cap);
  free(c);
  return cnt;
}

/* Depolarizing faults: linear indices L (ascending) over the active
 * positions and their types (a | b << 2, see the header). */
static int sample_depol(const orc_cfg *c, uint64_t seed, uint32_t traj,
                        uint32_t *L, uint8_t *type, int cap) {
  uint64_t S = c->dep_off[c->T];
  if (c->eps <= 0.0 || S == 0)
    return 0;
  static const uint8_t weyl[8][2] = {{0, 1}, {0, 2}, {1, 0}, {1, 1},
                                     {1, 2}, {2, 0}, {2, 1}, {2, 2}};
  static const uint8_t pauli[3][2] = {{1, 0}, {0, 1}, {1, 1}};
  uint64_t nb = (S + 63) / 64;
  int cnt = 0;
  int s = 1;
  for (uint64_t b = 0; b < nb; ++b) {
    uint64_t len = S - 64 * b < 64 ? S - 64 * b : 64;
    uint64_t pos = 0;
    for (uint32_t j = 0;; ++j) {
      uint32_t w[4];
      draw_words(seed, (uint32_t)b, j, traj, ORC_TAG_DEPOL, w);
      uint64_t u = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
      int o = 0;
      while (o < 64 && !(u < c->Gp[o]))
        ++o;
      if (o == 64 || pos + (uint64_t)o >= len)
        break;
      uint64_t Lx = 64 * b + pos + (uint64_t)o;
      while (c->dep_off[s + 1] <= Lx)
        ++s;
      int q = (int)(Lx - c->dep_off[s]);
      int router3 = c->enc == ORC_QUTRIT && (q & 1) == 0;
      const uint8_t *ab = router3 ? weyl[((uint64_t)w[2] * 8u) >> 32]
                                  : pauli[((uint64_t)w[2] * 3u) >> 32];
      if (cnt < cap && L) {
        L[cnt] = (uint32_t)Lx;
        type[cnt] = (uint8_t)(ab[0] | (ab[1] << 2));
      }
      ++cnt;
      pos += (uint64_t)o + 1;
    }
  }
  return cnt;
}

/* Slice and site of a depolarizing linear index. */
static void depol_site(const orc_cfg *c, uint32_t Lx, int *s, int *q) {
  int ss = 1;
  while (c->dep_off[ss + 1] <= Lx)
    ++ss;
  *s = ss;
  *q = (int)(Lx - c->dep_off[ss]);
}

int orc_sample_depol(int n, int k, int enc, double eps, uint64_t seed,
                     uint32_t traj, uint32_t *L, uint8_t *type, int cap) {
  static const uint32_t zero_mem[1] = {0};
  orc_cfg *c = (orc_cfg *)calloc(1, sizeof(orc_cfg));
  int rc = cfg_init(c, n, k, enc, 0.0, zero_mem);
  if (!rc)
    rc = cfg_extras(c, eps, NULL, NULL, NULL, -1);
  if (rc) {
    cfg_free(c);
    return rc;
  }
  int cnt = sample_depol(c, seed, traj, L, type, cap);
  cfg_free(c);
  return cnt;
}

/* Active positions per slice (for the tests): nact[s] for s = 0..T-1. */
int orc_depol_active(int n, int k, int *nact) {
  static const uint32_t zero_mem[1] = {0};
  orc_cfg *c = (orc_cfg *)calloc(1, sizeof(orc_cfg));
  int rc = cfg_init(c, n, k, ORC_QUBIT, 0.0, zero_mem);
  if (!rc)
    rc = cfg_extras(c, 0.0, NULL, NULL, NULL, -1);
  if (rc) {
    cfg_free(c);
    return rc;
  }
  for (int s = 0; s < c->T; ++s)
    nact[s] = c->nact[s];
  int T = c->T;
  cfg_free(c);
  return T;
}

/* ------------------------------------------------------------------------ */
/* Marking rule (Eq. subtree, Eq. badrange; Alg. 1 steps 1-2).              */
/* ------------------------------------------------------------------------ */
/* The node whose subtree is the bad range of a fault at node v. */
static uint32_t range_node(int enc, uint32_t v) {
  if (enc == ORC_QUTRIT)
    return v; /* Eq. subtree */
  /* Eq. badrange: a right child or a child of the root marks its own
   * subtree, a left child inherits the range of its parent, the root marks
   * everything. */
  for (;;) {
    if (v == 0)
      return 0;
    if (v <= 2)
      return v;
    if ((v & 1u) == 0)
      return v;
    v = (v - 1) >> 1;
  }
}

/* bad[i] = 1 if address i lies in the bad range of some candidate or of
 * some depolarizing fault (dsites: their tree sites; the rule is the same
 * whatever the fault's type, Sec. III B). */
static int classify_all(const orc_cfg *c, const uint32_t *L, int ncand,
                        const int *dsites, int ndep, uint8_t *bad) {
  int n = c->n;
  uint32_t nodes = (uint32_t)c->D - 1;
  uint8_t *mark = (uint8_t *)calloc(nodes, 1);
  for (int j = 0; j < ncand; ++j) {
    uint32_t q = L[j] % (uint32_t)c->M;
    mark[range_node(c->enc, q >> 1)] = 1;
  }
  for (int j = 0; j < ndep; ++j)
    mark[range_node(c->enc, (uint32_t)dsites[j] >> 1)] = 1;
  int nbad = 0;
  for (uint32_t i = 0; i < (uint32_t)c->D; ++i) {
    int b = 0;
    for (int l = 0; l < n && !b; ++l) {
      uint32_t v = ((uint32_t)1 << l) - 1 + (i >> (n - l));
      if (mark[v])
        b = 1;
    }
    bad[i] = (uint8_t)b;
    nbad += b;
  }
  free(mark);
  return nbad;
}

static int classify(const orc_cfg *c, const uint32_t *L, int ncand,
                    uint8_t *bad) {
  return classify_all(c, L, ncand, NULL, 0, bad);
}

int orc_classify(int n, int k, int enc, const uint32_t *L, int ncand,
                 uint8_t *bad) {
  static const uint32_t zero_mem[1] = {0};
  orc_cfg *c = (orc_cfg *)calloc(1, sizeof(orc_cfg));
  int rc = cfg_init(c, n, k, enc, 0.0, zero_mem);
  if (rc) {
    free(c);
    return rc;
  }
  int nb = classify(c, L, ncand, bad);
  free(c);
  return nb;
}

/* Range node of a site's fault, exported for the marking-rule tests. */
int orc_range_node(int enc, uint32_t v) { return (int)range_node(enc, v); }

/* ------------------------------------------------------------------------ */
/* Sparse state: one entry per component (address, bus word, tree levels).  */
/* Gates are permutations of basis labels, so components never split; the  */
/* state is kept as an array in initial-label order.                        */
/* ------------------------------------------------------------------------ */
typedef struct {
  int E, M;
  uint32_t *addr;
  uint32_t *bus;
  uint8_t *alive;
  int *nexc; /* number of excited tree sites */
  double complex *amp;
  uint8_t *tree; /* E x M levels */
} orc_state;

static int state_alloc(orc_state *st, int E, int M) {
  st->E = E;
  st->M = M;
  st->addr = (uint32_t *)malloc(sizeof(uint32_t) * E);
  st->bus = (uint32_t *)malloc(sizeof(uint32_t) * E);
  st->alive = (uint8_t *)malloc(E);
  st->nexc = (int *)malloc(sizeof(int) * E);
  st->amp = (double complex *)malloc(sizeof(double complex) * E);
  st->tree = (uint8_t *)malloc((size_t)E * (size_t)M);
  return st->addr && st->bus && st->alive && st->nexc && st->amp && st->tree
             ? 0
             : -2;
}

static void state_free(orc_state *st) {
  free(st->addr);
  free(st->bus);
  free(st->alive);
  free(st->nexc);
  free(st->amp);
  free(st->tree);
}

/* The input state after the first wall.  The data-loading input has
 * uniform address amplitudes and bus word 0; a general input sum_i c_i
 * |i>|j_i> or sum_ij c_ij |i>|j> (Sec. IV D).  For the qubit encoding the
 * first Hadamard wall acts on the noiseless bus before any tree gate touches
 * it, so it is applied here: component (i, beta) starts with amplitude
 * 2^(-k/2) sum_j c_ij (-1)^(beta . j) (j ascending), alive when the input
 * holds address i.  The qutrit encoding carries the bus word in the
 * computational basis: one component per address (bus word j_i), or with
 * c_ij one per (address, bus word), alive when its amplitude is nonzero. */
static void state_init(const orc_cfg *c, orc_state *st) {
  double wall = c->enc == ORC_QUBIT ? 1.0 / sqrt((double)c->K2) : 1.0;
  for (int x = 0; x < c->E; ++x) {
    memset(st->tree + (size_t)x * c->M, 0, c->M);
    st->nexc[x] = 0;
    if (c->enc == ORC_QUBIT) {
      uint32_t i = (uint32_t)x >> c->k;
      uint32_t beta = (uint32_t)x & (uint32_t)(c->K2 - 1);
      double complex v = 0.0;
      if (c->cab) {
        for (int j = 0; j < c->K2; ++j) {
          double complex cj = c->cab[(size_t)i * c->K2 + j];
          v += (__builtin_popcount(beta & (uint32_t)j) & 1) ? -cj : cj;
        }
      } else {
        /* the first wall on |j_i>: sum_beta (-1)^(beta . j_i) |beta> */
        double complex ci = in_amp(c, i);
        v = (__builtin_popcount(beta & in_bus(c, i)) & 1) ? -ci : ci;
      }
      st->addr[x] = i;
      st->bus[x] = beta;
      st->amp[x] = v * wall;
      st->alive[x] = present(c, i);
    } else if (c->cab) {
      uint32_t i = (uint32_t)x / (uint32_t)c->K2;
      uint32_t j = (uint32_t)x % (uint32_t)c->K2;
      st->addr[x] = i;
      st->bus[x] = j;
      st->amp[x] = c->cab[x];
      st->alive[x] = c->cab[x] != 0.0;
    } else {
      double complex ci = in_amp(c, (uint32_t)x);
      st->addr[x] = (uint32_t)x;
      st->bus[x] = in_bus(c, (uint32_t)x);
      st->amp[x] = ci;
      st->alive[x] = ci != 0.0;
    }
  }
}

/* One depolarizing fault (a, b) on site q of component x: level v becomes
 * v + a (mod d), then the amplitude takes w_d^(b (v + a)). */
static void apply_depol(const orc_cfg *c, orc_state *st, int x, int q,
                        int a, int b) {
  uint8_t *tr = st->tree + (size_t)x * c->M;
  int d = (c->enc == ORC_QUTRIT && (q & 1) == 0) ? 3 : 2;
  int v = tr[q];
  int w = (v + a) % d;
  tr[q] = (uint8_t)w;
  st->nexc[x] += (w != 0) - (v != 0);
  int ph = (b * w) % d;
  if (ph == 0)
    return;
  if (d == 2) {
    st->amp[x] = -st->amp[x];
  } else {
    const double complex w3 = -0.5 + I * (sqrt(3.0) / 2.0);
    st->amp[x] *= ph == 1 ? w3 : conj(w3);
  }
}

static void swap_u8(uint8_t *a, uint8_t *b) {
  uint8_t t = *a;
  *a = *b;
  *b = t;
}

/* Apply one scheduled event to component x. */
static void apply_event(const orc_cfg *c, orc_state *st, int x, int type,
                        int arg) {
  uint8_t *tr = st->tree + (size_t)x * c->M;
  int n = c->n;
  switch (type) {
  case EV_COPY: { /* CNOT from address bit t into the root data slot */
    uint32_t bit = (st->addr[x] >> (n - 1 - arg)) & 1u;
    if (bit) {
      tr[1] ^= 1;
      st->nexc[x] += tr[1] ? 1 : -1;
    }
    break;
  }
  case EV_STORE: {
    int l = arg;
    uint32_t v0 = ((uint32_t)1 << l) - 1, v1 = ((uint32_t)2 << l) - 1;
    for (uint32_t v = v0; v < v1; ++v) {
      uint8_t *r = &tr[2 * v], *d = &tr[2 * v + 1];
      if (c->enc == ORC_QUBIT) {
        swap_u8(r, d); /* SWAP(a_v, d_v) */
      } else {
        int gated;
        if (v == 0) {
          gated = 1;
        } else {
          uint32_t p = (v - 1) >> 1;
          gated = (v & 1u) ? tr[2 * p] == LV_L : tr[2 * p] == LV_R;
        }
        if (!gated)
          continue;
        /* (W,0)<->(L,0), (W,1)<->(R,0); (L,1),(R,1) unchanged */
        if (*r == LV_W) {
          uint8_t b = *d;
          *r = b ? LV_R : LV_L;
          *d = 0;
          if (!b)
            st->nexc[x] += 1;
        } else if (*d == 0) {
          uint8_t b = *r == LV_R ? 1 : 0;
          *r = LV_W;
          *d = b;
          if (!b)
            st->nexc[x] -= 1;
        }
      }
    }
    break;
  }
  case EV_CSWAP: {
    int l = arg;
    uint32_t v0 = ((uint32_t)1 << l) - 1, v1 = ((uint32_t)2 << l) - 1;
    for (uint32_t v = v0; v < v1; ++v) {
      uint8_t r = tr[2 * v];
      uint32_t ch;
      if (c->enc == ORC_QUBIT) {
        ch = r ? 2 * v + 2 : 2 * v + 1;
      } else {
        if (r == LV_W)
          continue; /* the wait state blocks routing */
        ch = r == LV_L ? 2 * v + 1 : 2 * v + 2;
      }
      swap_u8(&tr[2 * v + 1], &tr[2 * ch + 1]);
    }
    break;
  }
  case EV_BUS: { /* SWAP(bus_b, d_0) */
    uint32_t bb = (st->bus[x] >> arg) & 1u;
    uint8_t d = tr[1];
    tr[1] = (uint8_t)bb;
    st->bus[x] = (st->bus[x] & ~(1u << arg)) | ((uint32_t)d << arg);
    st->nexc[x] += (int)bb - (int)d;
    break;
  }
  case EV_FETCH: {
    int l = n - 1;
    uint32_t v0 = ((uint32_t)1 << l) - 1, v1 = ((uint32_t)2 << l) - 1;
    for (uint32_t v = v0; v < v1; ++v) {
      uint32_t p = v - v0;
      uint8_t r = tr[2 * v];
      if (c->enc == ORC_QUBIT) {
        /* CZ phase kickback: -1 on d_v = 1 when the routed cell holds 1 */
        if (tr[2 * v + 1]) {
          uint32_t cell = 2 * p + (r ? 1u : 0u);
          if ((c->mem[cell] >> arg) & 1u)
            st->amp[x] = -st->amp[x];
        }
      } else {
        /* computational-basis CNOT from the routed cell */
        if (r == LV_W)
          continue;
        uint32_t cell = 2 * p + (r == LV_R ? 1u : 0u);
        if ((c->mem[cell] >> arg) & 1u) {
          tr[2 * v + 1] ^= 1;
          st->nexc[x] += tr[2 * v + 1] ? 1 : -1;
        }
      }
    }
    break;
  }
  default:
    break;
  }
}

/* Neumaier compensated sum. */
typedef struct {
  double s, c;
} nsum;
static void nadd(nsum *a, double v) {
  double t = a->s + v;
  if (fabs(a->s) >= fabs(v))
    a->c += (a->s - t) + v;
  else
    a->c += (v - t) + a->s;
  a->s = t;
}
static double nval(const nsum *a) { return a->s + a->c; }

static double abs2(double complex z) {
  return creal(z) * creal(z) + cimag(z) * cimag(z);
}

typedef struct {
  /* per-trajectory results */
  double fid, fid_pre;
  double w_ground, w_total;
  int ncand, nbad, ref, nexplicit;
  int njumps, first_jump;
  int ref_survived, q_ground;
  int max_exc;
  int ndep; /* depolarizing faults of the trajectory */
} orc_result;

#define ORC_JLOG_MAX 4096

typedef struct {
  int n;                     /* entries used */
  int slice[ORC_JLOG_MAX];   /* slice of the jump */
  int site[ORC_JLOG_MAX];    /* tree site */
  int level[ORC_JLOG_MAX];   /* 1 = qubit/L/data, 2 = R */
} orc_jlog;

/* One joint damping layer (Eq. layerkraus, Theorem 4, Eq. maskweight). */
static int damping_layer(const orc_cfg *c, orc_state *st, int s,
                         const int *cq, int nc, double uaux, orc_jlog *jl,
                         int *jsite, int *jlev) {
  int nJ = 0;
  if (nc > 0) {
    int any = 0;
    for (int x = 0; x < st->E && !any; ++x) {
      if (!st->alive[x])
        continue;
      const uint8_t *tr = st->tree + (size_t)x * c->M;
      for (int j = 0; j < nc; ++j)
        if (tr[cq[j]]) {
          any = 1;
          break;
        }
    }
    if (any) {
      nsum we = {0, 0}, wn = {0, 0};
      for (int x = 0; x < st->E; ++x) {
        if (!st->alive[x])
          continue;
        const uint8_t *tr = st->tree + (size_t)x * c->M;
        int hit = 0;
        for (int j = 0; j < nc; ++j)
          if (tr[cq[j]])
            hit = 1;
        if (hit)
          nadd(&wn, abs2(st->amp[x]));
        else
          nadd(&we, abs2(st->amp[x]));
      }
      double w_empty = nval(&we), w_ne = nval(&wn);
      double r = uaux * (w_empty + w_ne);
      if (!(r < w_empty)) {
        double r2 = r - w_empty, cum = 0.0;
        int pick = -1, last = -1;
        for (int x = 0; x < st->E; ++x) {
          if (!st->alive[x])
            continue;
          const uint8_t *tr = st->tree + (size_t)x * c->M;
          int hit = 0;
          for (int j = 0; j < nc; ++j)
            if (tr[cq[j]])
              hit = 1;
          if (!hit)
            continue;
          last = x;
          cum += abs2(st->amp[x]);
          if (cum > r2) {
            pick = x;
            break;
          }
        }
        if (pick < 0)
          pick = last;
        const uint8_t *tr = st->tree + (size_t)pick * c->M;
        for (int j = 0; j < nc; ++j)
          if (tr[cq[j]]) {
            jsite[nJ] = cq[j];
            jlev[nJ] = tr[cq[j]];
            ++nJ;
          }
      }
    }
  }
  /* K_J = prod_{q in J} K1_q prod_{q not in J} K0_q on every component */
  for (int x = 0; x < st->E; ++x) {
    if (!st->alive[x])
      continue;
    uint8_t *tr = st->tree + (size_t)x * c->M;
    int ok = 1;
    for (int j = 0; j < nJ; ++j)
      if (tr[jsite[j]] != jlev[j])
        ok = 0;
    if (!ok) {
      st->alive[x] = 0;
      continue;
    }
    double complex f = 1.0;
    for (int j = 0; j < nJ; ++j)
      f *= c->sg;
    for (int e = 0; e < st->nexc[x] - nJ; ++e)
      f *= c->a;
    st->amp[x] *= f;
    for (int j = 0; j < nJ; ++j)
      tr[jsite[j]] = 0;
    st->nexc[x] -= nJ;
  }
  if (jl)
    for (int j = 0; j < nJ && jl->n < ORC_JLOG_MAX; ++j) {
      jl->slice[jl->n] = s;
      jl->site[jl->n] = jsite[j];
      jl->level[jl->n] = jlev[j];
      jl->n++;
    }
  return nJ;
}

static int count_exc(const orc_cfg *c, const orc_state *st, int x) {
  const uint8_t *tr = st->tree + (size_t)x * c->M;
  int m = 0;
  for (int q = 0; q < c->M; ++q)
    m += tr[q] != 0;
  return m;
}

/* History source: sampled from the seed, or forced by the caller. */
typedef struct {
  const uint32_t *L; /* forced candidates (ascending), or NULL */
  int ncand;
  const double *uaux; /* forced auxiliary uniforms indexed by slice, or NULL */
  double ufin;        /* forced final uniform if >= 0 */
  int dep_forced;     /* 1: the depolarizing faults below replace the draws */
  const uint32_t *dS; /* forced depolarizing faults: slices (ascending), */
  const uint32_t *dQ; /* sites (any site of the tree), */
  const uint8_t *dtype; /* and types (a | b << 2) */
  int ndep;
} orc_forced;

/* Evolve one trajectory; optionally stop after the gates of slice
 * stop_slice (> 0) and leave the state in st. */
static int run_traj(const orc_cfg *c, uint64_t seed, uint32_t traj,
                    const orc_forced *fh, int check_counts, orc_state *st,
                    orc_result *res, orc_jlog *jl) {
  int T = c->T, M = c->M;
  uint32_t *L = NULL;
  int ncand;
  if (fh && fh->L) {
    ncand = fh->ncand;
    L = (uint32_t *)malloc(sizeof(uint32_t) * (ncand > 0 ? ncand : 1));
    memcpy(L, fh->L, sizeof(uint32_t) * ncand);
  } else {
    ncand = sample_candidates(c, seed, traj, NULL, 0);
    L = (uint32_t *)malloc(sizeof(uint32_t) * (ncand > 0 ? ncand : 1));
    sample_candidates(c, seed, traj, L, ncand);
  }
  /* depolarizing faults: sampled, or forced */
  int ndep;
  uint32_t *dL = NULL;
  uint8_t *dty;
  int *dslice, *dsite;
  if (fh && fh->dep_forced) {
    ndep = fh->ndep;
    dty = (uint8_t *)malloc(ndep > 0 ? ndep : 1);
    dslice = (int *)malloc(sizeof(int) * (ndep > 0 ? ndep : 1));
    dsite = (int *)malloc(sizeof(int) * (ndep > 0 ? ndep : 1));
    for (int j = 0; j < ndep; ++j) {
      dslice[j] = (int)fh->dS[j];
      dsite[j] = (int)fh->dQ[j];
      dty[j] = fh->dtype[j];
    }
  } else {
    ndep = sample_depol(c, seed, traj, NULL, NULL, 0);
    dL = (uint32_t *)malloc(sizeof(uint32_t) * (ndep > 0 ? ndep : 1));
    dty = (uint8_t *)malloc(ndep > 0 ? ndep : 1);
    sample_depol(c, seed, traj, dL, dty, ndep);
    dslice = (int *)malloc(sizeof(int) * (ndep > 0 ? ndep : 1));
    dsite = (int *)malloc(sizeof(int) * (ndep > 0 ? ndep : 1));
    for (int j = 0; j < ndep; ++j)
      depol_site(c, dL[j], &dslice[j], &dsite[j]);
  }
  uint8_t *bad = (uint8_t *)malloc(c->D);
  int nbad = classify_all(c, L, ncand, dsite, ndep, bad);
  /* the reference: the smallest good address the input holds (with a
   * c_ij input, the smallest holding one bus word: a single branch) */
  int ref = -1;
  for (int i = 0; i < c->D; ++i)
    if (!bad[i] && present(c, (uint32_t)i) && (!c->cab || c->single[i])) {
      ref = i;
      break;
    }
  state_init(c, st);
  if (jl)
    jl->n = 0;
  int *cq = (int *)malloc(sizeof(int) * (ncand > 0 ? ncand : 1));
  int *jsite = (int *)malloc(sizeof(int) * (ncand > 0 ? ncand : 1));
  int *jlev = (int *)malloc(sizeof(int) * (ncand > 0 ? ncand : 1));
  int cpos = 0, njumps = 0, first_jump = 0, max_exc = 0, dpos = 0;
  for (int s = 1; s < T; ++s) {
    int d0 = dpos;
    while (dpos < ndep && dslice[dpos] == s)
      ++dpos;
    for (int x = 0; x < c->E; ++x) {
      if (!st->alive[x])
        continue;
      for (int e = 0; e < c->nev[s]; ++e)
        apply_event(c, st, x, c->ev_type[s][e], c->ev_arg[s][e]);
      for (int j = d0; j < dpos; ++j)
        apply_depol(c, st, x, dsite[j], dty[j] & 3, dty[j] >> 2);
      if (st->nexc[x] > max_exc)
        max_exc = st->nexc[x];
      if (check_counts && count_exc(c, st, x) != st->nexc[x])
        max_exc = 1 << 30; /* flags a bookkeeping error to the tests */
    }
    int nc = 0;
    while (cpos < ncand && (int)(L[cpos] / (uint32_t)M) + 1 == s)
      cq[nc++] = (int)(L[cpos++] % (uint32_t)M);
    double ua = (fh && fh->uaux) ? fh->uaux[s]
                                 : u53(draw_u64(seed, (uint32_t)s, 0, traj,
                                                ORC_TAG_AUX));
    int nJ = damping_layer(c, st, s, cq, nc, ua, jl, jsite, jlev);
    if (nJ > 0) {
      ++njumps;
      if (!first_jump)
        first_jump = s;
    }
  }
  free(cq);
  free(jsite);
  free(jlev);

  /* End of the query: wall 2 (qubit), tree measurement, fidelity.  The
   * ideal output is sum_ij c_ij |i>|j xor d_i>|ground>.  Ground components
   * of one address are grouped by bus word (after the wall, qubit); groups
   * with an excited tree are orthogonal to it and to each other.  With wmax,
   * the output words of the predicted good branches (good addresses other
   * than the reference) farther than wmax bit flips from their ideal word
   * are dropped (Sec. V). */
  double complex overlap = 0.0;
  nsum wg = {0, 0}, wt = {0, 0};
  {
    int K2 = c->K2;
    uint32_t kmask = (uint32_t)((1 << c->k) - 1);
    int per = c->E / c->D; /* components per address */
    double complex *grp = (double complex *)malloc(sizeof(double complex) * K2);
    double h = c->enc == ORC_QUBIT ? 1.0 / sqrt((double)K2) : 1.0;
    for (int i = 0; i < c->D; ++i) {
      int any = 0;
      for (int w = 0; w < K2; ++w)
        grp[w] = 0.0;
      for (int x = i * per; x < (i + 1) * per; ++x) {
        if (!st->alive[x])
          continue;
        if (st->nexc[x] != 0) {
          nadd(&wt, abs2(st->amp[x]));
          continue;
        }
        grp[st->bus[x] & kmask] += st->amp[x];
        any = 1;
      }
      if (!any)
        continue;
      int trunc = c->wmax >= 0 && c->enc == ORC_QUBIT && !bad[i] && i != ref &&
                  present(c, (uint32_t)i);
      uint32_t want = (single_bus(c, (uint32_t)i) ^ c->mem[i]) & kmask;
      for (int cw = 0; cw < K2; ++cw) {
        double complex v = 0.0;
        if (c->enc == ORC_QUBIT) {
          for (int beta = 0; beta < K2; ++beta)
            v += (__builtin_popcount((unsigned)(beta & cw)) & 1) ? -grp[beta]
                                                                 : grp[beta];
          v *= h;
        } else {
          v = grp[cw];
        }
        if (trunc && __builtin_popcount((unsigned)cw ^ want) > c->wmax)
          continue;
        nadd(&wg, abs2(v));
        overlap += conj(in_ab(c, (uint32_t)i, ((uint32_t)cw ^ c->mem[i]) & kmask)) * v;
      }
    }
    free(grp);
  }
  double w_ground = nval(&wg);
  double w_total = w_ground + nval(&wt);
  double uf = (fh && fh->ufin >= 0.0)
                  ? fh->ufin
                  : u53(draw_u64(seed, 0, 0, traj, ORC_TAG_FINAL));
  double r = uf * w_total;
  int q_ground = r < w_ground;
  double ov2 = abs2(overlap);
  res->fid = (q_ground && w_ground > 0.0) ? ov2 / w_ground : 0.0;
  res->fid_pre = w_total > 0.0 ? ov2 / w_total : 0.0;
  res->w_ground = w_ground;
  res->w_total = w_total;
  res->ncand = ncand;
  res->nbad = nbad;
  res->ref = ref;
  res->nexplicit = c->E;
  res->njumps = njumps;
  res->first_jump = first_jump;
  res->q_ground = q_ground;
  res->max_exc = max_exc;
  int rs = 0;
  if (ref >= 0)
    for (int x = 0; x < c->E; ++x)
      if (st->alive[x] && st->addr[x] == (uint32_t)ref)
        rs = 1;
  res->ref_survived = rs;
  res->ndep = ndep;
  free(bad);
  free(L);
  free(dL);
  free(dty);
  free(dslice);
  free(dsite);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Exported entry points (ctypes).                                          */
/* ------------------------------------------------------------------------ */

/* Result layout of orc_run_traj's double and int outputs. */
#define ORC_NRD 4
#define ORC_NRI 10

static void pack_result(const orc_result *r, double *rd, int *ri) {
  if (rd) {
    rd[0] = r->fid;
    rd[1] = r->fid_pre;
    rd[2] = r->w_ground;
    rd[3] = r->w_total;
  }
  if (ri) {
    ri[0] = r->ncand;
    ri[1] = r->nbad;
    ri[2] = r->ref;
    ri[3] = r->nexplicit;
    ri[4] = r->njumps;
    ri[5] = r->first_jump;
    ri[6] = r->ref_survived;
    ri[7] = r->q_ground;
    ri[8] = r->max_exc;
    ri[9] = r->ndep;
  }
}

/*
 * One trajectory.  forced_L/forced_ncand override the sampled candidates
 * when forced_L != NULL; forced_uaux (T entries, index = slice) overrides the
 * auxiliary uniforms; forced_ufin >= 0 overrides the final uniform.
 * Outputs: rd[ORC_NRD], ri[ORC_NRI]; optional jump log (jslice, jsite,
 * jlevel, capacity jcap, count in *njl); optional export of the final
 * pre-wall components (exp_cap entries): initial label (address * 2^k + bus
 * word for the qubit encoding, the address for the qutrit), address, bus
 * word, amplitude (re, im), and the sites/levels of each (M bytes per
 * component in exp_tree).  Returns the number of exported components, or < 0
 * on error.
 */
/*
 * The same with depolarizing faults of strength eps and a general input
 * (cin: 2 doubles per address or NULL; jin: bus word per address or NULL;
 * or cab: 2 doubles per (address, bus word), address-major, or NULL), and
 * the truncation wmax of the predicted good branches (-1: none).  With cab
 * the qutrit components are labelled address * 2^k + bus word.
 * dep_forced = 1 replaces the depolarizing draws by the faults
 * (dep_slice, dep_site, dep_type) [ndep], slices ascending, any site, types
 * a | b << 2.
 */
int orc_run_traj_ex(int n, int k, int enc, double gamma, double eps,
                    const uint32_t *mem, const double *cin, const uint32_t *jin,
                    const double *cab, int wmax,
                    uint64_t seed, uint32_t traj, const uint32_t *forced_L,
                    int forced_ncand, const double *forced_uaux,
                    double forced_ufin, int dep_forced,
                    const uint32_t *dep_slice, const uint32_t *dep_site,
                    const uint8_t *dep_type, int ndep, int check_counts,
                    double *rd, int *ri, int *jslice, int *jsite, int *jlevel,
                    int jcap, int *njl, uint32_t *exp_addr, uint32_t *exp_bus,
                    double *exp_amp, uint8_t *exp_tree, uint32_t *exp_label,
                    int exp_cap) {
  orc_cfg *c = (orc_cfg *)calloc(1, sizeof(orc_cfg));
  int rc = cfg_init(c, n, k, enc, gamma, mem);
  if (!rc)
    rc = cfg_extras(c, eps, cin, jin, cab, wmax);
  if (rc) {
    cfg_free(c);
    return rc;
  }
  orc_state st;
  if (state_alloc(&st, c->E, c->M)) {
    state_free(&st);
    cfg_free(c);
    return -2;
  }
  orc_forced fh = {forced_L, forced_ncand, forced_uaux, forced_ufin,
                   dep_forced, dep_slice, dep_site, dep_type, ndep};
  orc_jlog *jl = (orc_jlog *)malloc(sizeof(orc_jlog));
  orc_result res;
  run_traj(c, seed, traj, &fh, check_counts, &st, &res, jl);
  pack_result(&res, rd, ri);
  if (njl) {
    int m = jl->n < jcap ? jl->n : jcap;
    for (int j = 0; j < m; ++j) {
      jslice[j] = jl->slice[j];
      jsite[j] = jl->site[j];
      jlevel[j] = jl->level[j];
    }
    *njl = jl->n;
  }
  int ne = 0;
  if (exp_cap > 0) {
    for (int x = 0; x < c->E; ++x) {
      if (!st.alive[x])
        continue;
      if (ne < exp_cap) {
        exp_label[ne] = (uint32_t)x;
        exp_addr[ne] = st.addr[x];
        exp_bus[ne] = st.bus[x];
        exp_amp[2 * ne] = creal(st.amp[x]);
        exp_amp[2 * ne + 1] = cimag(st.amp[x]);
        memcpy(exp_tree + (size_t)ne * c->M, st.tree + (size_t)x * c->M, c->M);
      }
      ++ne;
    }
  }
  free(jl);
  state_free(&st);
  cfg_free(c);
  return ne;
}

int orc_run_traj(int n, int k, int enc, double gamma, const uint32_t *mem,
                 uint64_t seed, uint32_t traj, const uint32_t *forced_L,
                 int forced_ncand, const double *forced_uaux,
                 double forced_ufin, int check_counts, double *rd, int *ri,
                 int *jslice, int *jsite, int *jlevel, int jcap, int *njl,
                 uint32_t *exp_addr, uint32_t *exp_bus, double *exp_amp,
                 uint8_t *exp_tree, uint32_t *exp_label, int exp_cap) {
  return orc_run_traj_ex(n, k, enc, gamma, 0.0, mem, NULL, NULL, NULL, -1, seed, traj,
                         forced_L, forced_ncand, forced_uaux, forced_ufin, 0,
                         NULL, NULL, NULL, 0, check_counts, rd, ri, jslice, jsite,
                         jlevel, jcap, njl, exp_addr, exp_bus, exp_amp,
                         exp_tree, exp_label, exp_cap);
}

/*
 * Mask weights of one damping layer: evolve the forced history through the
 * damping layers of slices 1..s-1 and the gates of slice s, then return, for
 * the candidate sites cand[0..nc-1] of slice s, every distinct nonempty mask
 * J = C cap X(x) with its weight w(J) (Eq. maskweight) and w(empty).
 * Masks are returned as nc levels per entry (0 = not in J).
 */
int orc_layer_masks(int n, int k, int enc, double gamma, const uint32_t *mem,
                    const uint32_t *forced_L, int forced_ncand,
                    const double *forced_uaux, int s, const int *cand, int nc,
                    uint8_t *masks, double *weights, int cap, double *w_empty) {
  orc_cfg *c = (orc_cfg *)calloc(1, sizeof(orc_cfg));
  int rc = cfg_init(c, n, k, enc, gamma, mem);
  if (rc) {
    free(c);
    return rc;
  }
  orc_state st;
  state_alloc(&st, c->E, c->M);
  state_init(c, &st);
  int ncand = forced_ncand;
  int *cq = (int *)malloc(sizeof(int) * (ncand + 1));
  int *js = (int *)malloc(sizeof(int) * (ncand + 1));
  int *jv = (int *)malloc(sizeof(int) * (ncand + 1));
  int cpos = 0;
  for (int ss = 1; ss <= s; ++ss) {
    for (int x = 0; x < c->E; ++x) {
      if (!st.alive[x])
        continue;
      for (int e = 0; e < c->nev[ss]; ++e)
        apply_event(c, &st, x, c->ev_type[ss][e], c->ev_arg[ss][e]);
    }
    if (ss == s)
      break;
    int ncs = 0;
    while (cpos < ncand && (int)(forced_L[cpos] / (uint32_t)c->M) + 1 == ss)
      cq[ncs++] = (int)(forced_L[cpos++] % (uint32_t)c->M);
    damping_layer(c, &st, ss, cq, ncs, forced_uaux ? forced_uaux[ss] : 0.5,
                  NULL, js, jv);
  }
  int nm = 0;
  nsum we = {0, 0};
  uint8_t *cur = (uint8_t *)malloc(nc > 0 ? nc : 1);
  for (int x = 0; x < c->E; ++x) {
    if (!st.alive[x])
      continue;
    const uint8_t *tr = st.tree + (size_t)x * c->M;
    int hit = 0;
    for (int j = 0; j < nc; ++j) {
      cur[j] = tr[cand[j]];
      if (cur[j])
        hit = 1;
    }
    double w = abs2(st.amp[x]);
    if (!hit) {
      nadd(&we, w);
      continue;
    }
    int m;
    for (m = 0; m < nm; ++m)
      if (memcmp(masks + (size_t)m * nc, cur, nc) == 0)
        break;
    if (m == nm) {
      if (nm >= cap)
        continue;
      memcpy(masks + (size_t)m * nc, cur, nc);
      weights[m] = 0.0;
      ++nm;
    }
    weights[m] += w;
  }
  *w_empty = nval(&we);
  free(cur);
  free(cq);
  free(js);
  free(jv);
  state_free(&st);
  free(c);
  return nm;
}

/*
 * Batch of trajectories with OpenMP over trajectories: traj0 .. traj0+ntraj-1,
 * or the listed indices idx[0..ntraj-1] when idx is not NULL.  fid[ntraj],
 * fid_pre[ntraj] (or NULL), ri[ntraj*ORC_NRI] (or NULL).  nthreads <= 0 uses
 * the OpenMP default.  Returns the number of threads used.
 */
static int run_many(int n, int k, int enc, double gamma, double eps,
                    const uint32_t *mem, const double *cin, const uint32_t *jin,
                    const double *cab, int wmax, uint64_t seed, uint32_t traj0,
                    const uint32_t *idx, int ntraj, int nthreads, double *fid,
                    double *fid_pre, int *ri);

int orc_run_batch(int n, int k, int enc, double gamma, const uint32_t *mem,
                  uint64_t seed, uint32_t traj0, int ntraj, int nthreads,
                  double *fid, double *fid_pre, int *ri) {
  return run_many(n, k, enc, gamma, 0.0, mem, NULL, NULL, NULL, -1, seed,
                  traj0, NULL, ntraj, nthreads, fid, fid_pre, ri);
}

int orc_run_indices(int n, int k, int enc, double gamma, const uint32_t *mem,
                    uint64_t seed, const uint32_t *idx, int nidx, int nthreads,
                    double *fid, double *fid_pre, int *ri) {
  return run_many(n, k, enc, gamma, 0.0, mem, NULL, NULL, NULL, -1, seed, 0,
                  idx, nidx, nthreads, fid, fid_pre, ri);
}

/* Batches with depolarizing faults and a general input (see
 * orc_run_traj_ex); idx may be NULL (then traj0 .. traj0+ntraj-1). */
int orc_run_many_ex(int n, int k, int enc, double gamma, double eps,
                    const uint32_t *mem, const double *cin, const uint32_t *jin,
                    const double *cab, int wmax, uint64_t seed, uint32_t traj0,
                    const uint32_t *idx, int ntraj, int nthreads, double *fid,
                    double *fid_pre, int *ri) {
  return run_many(n, k, enc, gamma, eps, mem, cin, jin, cab, wmax, seed, traj0,
                  idx, ntraj, nthreads, fid, fid_pre, ri);
}

static int run_many(int n, int k, int enc, double gamma, double eps,
                    const uint32_t *mem, const double *cin, const uint32_t *jin,
                    const double *cab, int wmax, uint64_t seed, uint32_t traj0,
                    const uint32_t *idx, int ntraj, int nthreads, double *fid,
                    double *fid_pre, int *ri) {
  orc_cfg *c = (orc_cfg *)calloc(1, sizeof(orc_cfg));
  int rc = cfg_init(c, n, k, enc, gamma, mem);
  if (!rc)
    rc = cfg_extras(c, eps, cin, jin, cab, wmax);
  if (rc) {
    cfg_free(c);
    return rc;
  }
  int used = 1;
#ifdef _OPENMP
  if (nthreads > 0)
    omp_set_num_threads(nthreads);
#pragma omp parallel
  {
#pragma omp single
    used = omp_get_num_threads();
    orc_state st;
    state_alloc(&st, c->E, c->M);
#pragma omp for schedule(dynamic, 1)
    for (int t = 0; t < ntraj; ++t) {
      orc_result res;
      run_traj(c, seed, idx ? idx[t] : traj0 + (uint32_t)t, NULL, 0, &st, &res,
               NULL);
      fid[t] = res.fid;
      if (fid_pre)
        fid_pre[t] = res.fid_pre;
      if (ri)
        pack_result(&res, NULL, ri + (size_t)t * ORC_NRI);
    }
    state_free(&st);
  }
#else
  (void)nthreads;
  orc_state st;
  state_alloc(&st, c->E, c->M);
  for (int t = 0; t < ntraj; ++t) {
    orc_result res;
    run_traj(c, seed, idx ? idx[t] : traj0 + (uint32_t)t, NULL, 0, &st, &res,
             NULL);
    fid[t] = res.fid;
    if (fid_pre)
      fid_pre[t] = res.fid_pre;
    if (ri)
      pack_result(&res, NULL, ri + (size_t)t * ORC_NRI);
  }
  state_free(&st);
#endif
  cfg_free(c);
  return used;
}
