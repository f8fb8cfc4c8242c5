// Host side of the HIP library: contexts, schedule tables, work buffers,
// launch plans, autotuner and the C ABI declared in include/qram.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "qram_internal.h"

using namespace qr;

namespace {
thread_local std::string g_create_error;
}  // namespace

// One bucket of the evolution: trajectories with at most `emax` explicit
// components, run by `grid` persistent workgroups of `threads` threads, each
// thread holding `apt` addresses (apt * K2 component slots).
struct BucketShape {
  uint32_t emax = 0;
  int threads = 64;
  uint32_t apt = 1;
  uint32_t e_cap = 0;
  bool state_lds = false;
  uint32_t lds = 0;
  uint32_t grid = 1;
};

struct Plan {
  int nb = 0;
  BucketShape b[MAXB];
  bool persistent = true;
  uint32_t pool_slots = 0;  // max emax over buckets
  bool cdec_all = false;    // all candidates decoded into shared memory
  uint32_t cdec_cap = 0;    // decoded-candidate entries in shared memory
  uint32_t grid_max = 0;
  uint32_t ecap_max = 0;
  // plain full evolution: one launch of `grid` workgroups, grid-stride over
  // the batch's trajectories
  bool plain = false;
  // the plain engine's launch (plain plans, and the plain half of a split
  // plan): workgroup shape in pb, shared memory per workgroup
  BucketShape pb{};
  uint32_t plds = 0;
  uint32_t pslab = 0;  // words of each thread's record slab in shared memory (0: none)
  int pvar = 0;        // the plain kernel's register budget (plain_variant)
  // split plan (pruned mode with depolarizing noise on the data-loading
  // input): the trajectory kernel's buckets take the trajectories without a
  // depolarizing fault, the plain engine the others
  bool split = false;
};

struct qram_ctx {
  int n = 0, k = 0, enc = 0;
  double gamma = 0.0;
  double eps = 0.0;       // depolarizing strength
  bool general = false;   // depolarizing noise or a general input: the plain engine runs every mode
  bool dsplit = false;    // depolarizing noise only: pruned runs split by whether a trajectory drew a fault
  double *dcin = nullptr;  // general input amplitudes (device)
  uint32_t *djin = nullptr;
  double *dcab = nullptr, *dcamp = nullptr;  // pair amplitudes, component amplitudes
  uint8_t *daflag = nullptr;
  // the input as (address << 8 | bus word, normalised amplitude) pairs, for
  // the dense cross-check
  std::vector<uint32_t> in_idx;
  std::vector<double> in_amp;
  uint32_t *dep = nullptr, *ndep = nullptr;  // depolarizing faults of a batch
  uint32_t dep_cap = 0;
  int T = 0, M = 0, D = 0, K2 = 1, Emax = 0, lmax = 0, emax = 0, rec = 0;
  int device = 0, num_cu = 0;
  size_t lds_max = 0;
  hipStream_t stream = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  Tables htab{};
  Tables *dtab = nullptr;
  uint32_t *dmem = nullptr;
  double *dwpow = nullptr, *dapow = nullptr, *dftab = nullptr, *dctot = nullptr;
  std::vector<uint32_t> mem;
  std::string err;
  // work buffers (grown on demand)
  uint32_t batch_cap = 0;   // trajectories per batch the buffers hold
  uint32_t cand_cap = 0;    // candidate slots per trajectory
  size_t gstate_cap = 0;    // tier-1 words in gstate
  size_t pool_cap = 0;      // uint16 words in pool
  size_t devl_cap = 0;      // uint16 words in devl
  uint32_t *cand = nullptr, *ncand = nullptr, *nbad = nullptr, *ref = nullptr;
  uint32_t *nexpl = nullptr, *order = nullptr, *counter = nullptr, *errw = nullptr;
  uint32_t *bucket_base = nullptr;
  uint64_t *badbits = nullptr, *digest = nullptr;
  uint16_t *xlist = nullptr, *pool = nullptr;
  uint32_t *devl = nullptr;
  uint32_t *gstate = nullptr;
  double *fid_tmp = nullptr, *uaux = nullptr;
  // test entries: component export and jump logs
  uint32_t *dexp = nullptr, *djlog = nullptr, *djn = nullptr;
  size_t dexp_cap = 0, djlog_cap = 0, djn_cap = 0;
  double *dexpamp = nullptr;
  size_t dexpamp_cap = 0;
  // plain engine: record length; launch shape per mode (full, pruned,
  // plain): workgroups per CU and threads per workgroup, 0 = automatic
  int prec = 0;
  int plain_per_cu[3] = {0, 0, 0};
  int plain_thr[3] = {0, 0, 0};
  int plain_used_thr[3] = {0, 0, 0};  // threads of the last plain launch per mode
  bool plain_glob[3] = {false, false, false};  // records worked on in device memory
  double *pamp = nullptr, *pgrp = nullptr;
  uint8_t *phit = nullptr;
  size_t pamp_cap = 0, pgrp_cap = 0, phit_cap = 0;
  qram_traj_stats *st_tmp = nullptr;
  uint32_t out_cap = 0;
  // launch choice per mode: slots per thread (0 = automatic), schedule
  int spt[3] = {0, 0, 0};
  int schedule[3] = {1, 1, 0};
  bool tier2_global = false;
  // graph mode: every batch is captured once into a graph and replayed;
  // the executable graph is updated in place for the next batch
  bool use_graph = false;
  // qubit encoding: damping candidates mark their own subtree (Eq. subtree)
  // instead of Eq. badrange
  bool mark_subtree = false;
  hipGraphExec_t gexec = nullptr;
  Run graph_run{};       // the arguments the executable graph was captured with
  uint64_t graph_sig = 0;  // launch-plan signature of the executable graph
  double last_ms[3] = {0, 0, 0};
  // stage timing of asynchronous runs: four events per batch
  bool timing = false;
  std::vector<hipEvent_t> tev;  // EVB per timed batch: 4 stage events, then 2 per bucket
  size_t tev_used = 0;
  uint32_t tev_launches = 0;  // evolution launches inside the timed batches
  std::vector<int> tev_nb;    // buckets of each timed batch
  uint32_t tev_emax[MAXB] = {0, 0, 0, 0, 0, 0};  // bucket bounds of the last timed batch
  // device address of this device's no-allocation scratch array (null if
  // it could not be resolved), and whether a no-allocation run used it
  unsigned char *scratch = nullptr;
  bool scratch_used = false;
};

// ---------------------------------------------------------------------------
// No-allocation runs.  Callers that cannot allocate device memory (work
// under graph capture, tight serving loops) run through
// qram_run_pruned_async_noalloc, whose work buffers live in this static
// array instead of context-owned allocations.  Each device holds its own
// copy until the process ends.  In host code the array's name is only a
// stand-in: its device address on each device comes from
// hipGetSymbolAddress, taken once per device in qram_create with that
// device current, and only that address is handed to kernels and copies.
// ---------------------------------------------------------------------------
constexpr size_t SCRATCH_BYTES = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

constexpr int SCRATCH_MAX_DEVICES = 64;
struct ScratchDev {
  std::once_flag once;
  void *ptr = nullptr;
  hipError_t err = hipSuccess;
};
ScratchDev g_scratch[SCRATCH_MAX_DEVICES];

// The scratch array's address on `device`, which must be current.
unsigned char *scratch_address(int device) {
  if (device < 0 || device >= SCRATCH_MAX_DEVICES) return nullptr;
  ScratchDev &d = g_scratch[device];
  std::call_once(d.once, [&d] {
    void *p = nullptr;
    d.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (d.err == hipSuccess)
      d.ptr = p;
    else
      (void)hipGetLastError();
  });
  return static_cast<unsigned char *>(d.ptr);
}

// Fixed header of the scratch array: error word, queue heads, bucket bases.
constexpr size_t SCR_ERR = 0, SCR_COUNTER = 256, SCR_BBASE = 512, SCR_HEAD = 1024;

}  // namespace

namespace {

qram_status fail(qram_ctx *c, qram_status st, const std::string &msg) {
  if (c)
    c->err = msg;
  else
    g_create_error = msg;
  return st;
}

#define HIPCHK(c, expr)                                                       \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess)                                                     \
      return fail((c), QRAM_E_DEVICE,                                         \
                  std::string(#expr) + ": " + hipGetErrorString(e_));         \
  } while (0)

template <typename T>
qram_status dev_alloc(qram_ctx *c, T **p, size_t count) {
  if (*p) {
    (void)hipFree(*p);
    *p = nullptr;
  }
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(c, QRAM_E_NOMEM, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed");
  }
  return QRAM_OK;
}

template <typename T>
void dev_free(T **p) {
  if (*p) (void)hipFree(*p);
  *p = nullptr;
}

// Device buffer of at least `count` elements, grown on demand.
template <typename T>
qram_status grow(qram_ctx *c, T **p, size_t *cap, size_t count) {
  if (count <= *cap && *p) return QRAM_OK;
  qram_status st = dev_alloc(c, p, count);
  *cap = st ? 0 : count;
  return st;
}

// ---------------------------------------------------------------------------
// Schedule tables.  Events follow the bucket-brigade query of Sec. II A:
// address bit t is copied into the root data slot at 2t+1, moves down one
// layer per slice and is stored into the router of layer t at 3t+2; data bit
// b enters at 2n+2b+1, is fetched at 3n+2b+1 and leaves at 4n+2b+1; every
// event has its mirror at T-s.  Token positions are then obtained by moving
// each token of one generic root-to-leaf path through these events.
// ---------------------------------------------------------------------------
bool build_tables(qram_ctx *c, std::string &why) {
  Tables &t = c->htab;
  std::memset(&t, 0, sizeof(t));
  const int n = c->n, k = c->k, T = c->T;
  t.n = n;
  t.k = k;
  t.enc = c->enc;
  t.T = T;
  t.M = c->M;
  t.D = c->D;
  t.K2 = c->K2;
  t.lmax = c->lmax;
  t.sg = std::sqrt(c->gamma);
  t.emax = c->emax;
  t.rec = c->rec;
  // geometric-walk thresholds: G[o] = floor(2^64 (1 - (1-p)^(o+1))), for
  // the damping candidates (p = gamma) and the depolarizing faults (p = eps)
  auto thresholds = [](double p, uint64_t *G) {
    const double q = 1.0 - p;
    double qp = 1.0;
    for (int o = 0; o < 64; ++o) {
      qp = qp * q;
      const double x = std::ldexp(1.0 - qp, 64);
      G[o] = x >= 18446744073709551616.0 ? UINT64_MAX : (uint64_t)x;
    }
  };
  thresholds(c->gamma, t.G);
  thresholds(c->eps, t.Gp);
  // depolarizing placement (App. C): in slice s every site of the layers
  // above the leaf layer whose router holds its address bit both before and
  // after the gates of s (stored at 3t+2, unstored at T-3t-2)
  t.depol = c->eps > 0.0 ? 1 : 0;
  {
    uint32_t off = 0;
    for (int sl = 0; sl <= MAXT; ++sl) t.dep_off[sl] = 0;
    for (int sl = 1; sl < T; ++sl) {
      int l = 0;
      for (int tt = 0; tt + 1 < c->n; ++tt)
        if (3 * tt + 2 < sl && sl < T - 3 * tt - 2) ++l;
      t.dep_off[sl] = off;
      off += 2u * ((1u << l) - 1u);
    }
    t.dep_off[T] = off;
  }
  t.cin = nullptr;
  t.jin = nullptr;
  for (int s = 0; s < MAXT; ++s) {
    t.copy_t[s] = t.store_l[s] = t.bus_b[s] = t.fetch_b[s] = -1;
    t.cswap[s] = 0;
  }
  auto set1 = [&](int8_t *arr, int s, int v) -> bool {
    if (arr[s] != -1 && arr[s] != v) return false;
    arr[s] = (int8_t)v;
    return true;
  };
  bool ok = true;
  for (int a = 0; a < n; ++a) {
    ok &= set1(t.copy_t, 2 * a + 1, a);
    ok &= set1(t.copy_t, T - 2 * a - 1, a);
    ok &= set1(t.store_l, 3 * a + 2, a);
    ok &= set1(t.store_l, T - 3 * a - 2, a);
    for (int l = 0; l < a; ++l) {
      t.cswap[2 * a + 2 + l] |= 1u << l;
      t.cswap[T - 2 * a - 2 - l] |= 1u << l;
    }
  }
  for (int b = 0; b < k; ++b) {
    ok &= set1(t.bus_b, 2 * n + 2 * b + 1, b);
    ok &= set1(t.bus_b, 4 * n + 2 * b + 1, b);
    ok &= set1(t.fetch_b, 3 * n + 2 * b + 1, b);
    for (int l = 0; l + 1 < n; ++l) {
      t.cswap[2 * n + 2 * b + 2 + l] |= 1u << l;
      t.cswap[4 * n + 2 * b - l] |= 1u << l;
    }
  }
  if (!ok) {
    why = "schedule events collide";
    return false;
  }
  const int ntok = n + k;
  std::vector<int> pos(ntok, -1);  // layer << 1 | slot, -1 outside
  std::vector<int> entered(ntok, 0);
  for (int s = 1; s < T; ++s) {
    if (t.copy_t[s] >= 0) {
      const int a = t.copy_t[s];
      if (pos[a] < 0 && !entered[a]) {
        pos[a] = 1;  // root data slot
        entered[a] = 1;
      } else if (pos[a] == 1) {
        pos[a] = -1;
      } else {
        why = "address token not at the root when uncopied";
        return false;
      }
    }
    if (t.store_l[s] >= 0) {
      const int l = t.store_l[s];
      for (int x = 0; x < ntok; ++x)
        if (pos[x] >= 0 && (pos[x] >> 1) == l) pos[x] ^= 1;
    }
    if (t.cswap[s]) {
      for (int x = 0; x < ntok; ++x) {
        if (pos[x] < 0 || !(pos[x] & 1)) continue;
        const int l = pos[x] >> 1;
        if ((t.cswap[s] >> l) & 1u)
          pos[x] = ((l + 1) << 1) | 1;
        else if (l >= 1 && ((t.cswap[s] >> (l - 1)) & 1u))
          pos[x] = ((l - 1) << 1) | 1;
      }
    }
    if (t.bus_b[s] >= 0) {
      const int x = n + t.bus_b[s];
      if (pos[x] < 0 && !entered[x]) {
        pos[x] = 1;
        entered[x] = 1;
      } else if (pos[x] == 1) {
        pos[x] = -1;
      } else {
        why = "data token not at the root when it leaves";
        return false;
      }
    }
    for (int l = 0; l < MAXN; ++l) t.tok[s][l][0] = t.tok[s][l][1] = NONE;
    uint32_t am = 0, dm = 0;
    int nr = 0;
    for (int x = 0; x < ntok; ++x) {
      t.pos[s][x] = pos[x] < 0 ? NONE : (uint8_t)pos[x];
      if (pos[x] < 0) continue;
      const int l = pos[x] >> 1, slot = pos[x] & 1;
      if (l >= n) {
        why = "token below the leaf layer";
        return false;
      }
      if (t.tok[s][l][slot] != NONE) {
        why = "two tokens share a site of the path";
        return false;
      }
      t.tok[s][l][slot] = (uint8_t)x;
      if (x < n) {
        if (c->enc == QUBIT || slot == 1) am |= 1u << (n - 1 - x);
        if (c->enc == QUTRIT && slot == 0) ++nr;
      } else {
        const int b = x - n;
        if (c->enc == QUBIT || s >= 3 * n + 2 * b + 1) dm |= 1u << b;
      }
    }
    t.amask[s] = am;
    t.dmask[s] = dm;
    t.nrouter[s] = (uint8_t)nr;
    for (int a = 0; a < n; ++a)
      t.cntA[s][a] = (uint16_t)(t.cntA[s - 1][a] + ((am >> (n - 1 - a)) & 1u));
    for (int b = 0; b < k; ++b)
      t.cntD[s][b] = (uint16_t)(t.cntD[s - 1][b] + ((dm >> b) & 1u));
    t.cntR[s] = (uint16_t)(t.cntR[s - 1] + nr);
  }
  for (int x = 0; x < ntok; ++x)
    if (pos[x] >= 0) {
      why = "a token is still in the tree after the last slice";
      return false;
    }
  for (int s = T; s < MAXT; ++s) {
    for (int a = 0; a < n; ++a) t.cntA[s][a] = t.cntA[T - 1][a];
    for (int b = 0; b < k; ++b) t.cntD[s][b] = t.cntD[T - 1][b];
    t.cntR[s] = t.cntR[T - 1];
  }
  return true;
}

uint32_t cand_capacity(const qram_ctx *c) {
  const double S = (double)(c->T - 1) * (double)c->M;
  const double mean = S * c->gamma;
  const double sd = std::sqrt(S * c->gamma * (1.0 - c->gamma));
  double cap = mean + 10.0 * sd + 32.0;
  if (cap > S) cap = S;
  uint32_t r = (uint32_t)std::ceil(cap);
  return std::max<uint32_t>(r, 32u);
}

// Depolarizing faults per trajectory: mean + 10 sd over the active positions.
uint32_t dep_capacity(const qram_ctx *c) {
  if (c->eps <= 0.0) return 0;
  const double S = (double)c->htab.dep_off[c->T];
  double cap = S * c->eps + 10.0 * std::sqrt(S * c->eps * (1.0 - c->eps)) + 32.0;
  if (cap > S) cap = S;
  return std::max<uint32_t>((uint32_t)std::ceil(cap), 32u);
}

uint32_t pow2ceil(uint32_t x) {
  uint32_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Plain-engine launch shape of a mode: the caller's choice where one was set,
// else the automatic one.
// The automatic shape: as many workgroups per compute unit as fit (the
// engine waits on memory more than it computes), of 256 threads, or of 64 /
// 128 threads when a trajectory holds at most 256 components (pruned /
// full), so that small trajectories do not leave most lanes idle.
// A split pruned run's plain share is few trajectories, and its time is
// that of its longest ones (a fault near the root leaves nearly the whole
// tree bad), which one workgroup evolves alone: 256 threads, or 1024 when
// the batch's expected faulted trajectories are about as many as the
// device holds workgroups of 256 threads, at most ten per compute unit
// (ntraj trajectories, each drawing a fault with the context's
// probability; for a batch of unknown size, ntraj = 0, at most 60% of the
// trajectories drawing a fault stands in), and a trajectory holds at least
// 2048 components, two a thread.  With more faulted trajectories the share
// fills the device and smaller workgroups keep more of them in flight;
// with fewer components most of the threads idle.
void plain_shape(const qram_ctx *c, int mode, int &threads, int &per_cu, bool &glob, uint32_t ntraj) {
  const int m = mode;
  threads = c->plain_thr[m];
  const bool share = c->dsplit && mode == QRAM_MODE_PRUNED;
  if (!threads) {
    const double pf = share ? 1.0 - std::pow(1.0 - c->eps, (double)c->htab.dep_off[c->T]) : 1.0;
    const bool few = ntraj ? pf * (double)ntraj <= 10.0 * (double)c->num_cu : pf <= 0.6;
    if (share && c->Emax >= 2048 && few)
      threads = 1024;
    else
      threads = (c->Emax > 256 || share) ? PLAIN_THREADS : (mode == QRAM_MODE_PRUNED ? 64 : 128);
  }
  per_cu = c->plain_per_cu[m] ? c->plain_per_cu[m] : 32;  // (capped by occupancy)
  glob = c->plain_glob[m];
}

// The slabs' share of a workgroup's shared memory.  With depolarizing noise
// the record capacity counts every stray a trajectory may hold, so slabs
// are shorter than records and the budget decides how many workgroups a
// compute unit holds.  Qubit trajectories that draw few faults (their
// lists stay short) run faster with a smaller budget, which lets five
// workgroups of the 96-register build share a compute unit, than with
// longer slabs; many faults lengthen every list, and the larger budget
// keeps more of them in shared memory.  The qutrit kernel has no build
// that holds five, and keeps the larger budget.
constexpr uint32_t PLAIN_SLAB_FEW_FAULTS_BYTES = 26 * 1024;
constexpr double PLAIN_FEW_FAULTS = 32.0;  // expected faults per trajectory
uint32_t plain_slab_budget(const qram_ctx *c) {
  if (c->eps <= 0.0 || c->enc != QUBIT) return PLAIN_SLAB_BYTES;
  const double faults = c->eps * (double)c->htab.dep_off[c->T];
  return faults <= PLAIN_FEW_FAULTS ? PLAIN_SLAB_FEW_FAULTS_BYTES : PLAIN_SLAB_BYTES;
}

// Shared memory of a plain-engine workgroup of `threads`: the slice state,
// and a record slab per thread (words; 0 when the records stay in device
// memory: asked for, QRAM_OPT_TIER2_GLOBAL, or a slab within the budget
// that is shorter than both the record and 32 words).  A slab shorter than
// the record capacity takes the records that fit it.
uint32_t plain_slab(const qram_ctx *c, int threads, bool glob) {
  if (glob || c->tier2_global) return 0;
  // (workgroups of more than 256 threads, one or two per compute unit: 40
  // words a thread)
  const uint32_t budget = threads > 256 ? (uint32_t)threads * 80u : plain_slab_budget(c);
  const uint32_t sw = std::min<uint32_t>((uint32_t)c->prec, (budget / 2u / (uint32_t)threads) & ~7u);
  return (sw == (uint32_t)c->prec || sw >= 32u) ? sw : 0u;
}
uint32_t plain_lds(const qram_ctx *c, int threads, bool glob) {
  return plain_lds_bytes(c->M, (uint32_t)threads * plain_slab(c, threads, glob));
}

// Launch plan of a mode.  The full mode evolves every address, so it has one
// bucket.  The pruned mode's explicit work varies per trajectory (bad
// addresses plus the reference), so trajectories are grouped by it, each
// group with a workgroup size and LDS footprint sized for its largest member.
// The plain engine's launch of a mode (pl.pb, plds, pslab).
qram_status plain_plan(qram_ctx *c, int mode, uint32_t ntraj, Plan &pl) {
  int threads = 0, per_cu = 0;
  bool glob = false;
  plain_shape(c, mode, threads, per_cu, glob, ntraj);
  pl.plds = plain_lds(c, threads, glob);
  pl.pslab = plain_slab(c, threads, glob);
  int occ = 0;
  pl.pvar = plain_variant(c->enc, threads, pl.plds, per_cu, occ);
  if (occ < 1) return fail(c, QRAM_E_DEVICE, "plain engine: no workgroup fits a compute unit");
  per_cu = std::min(per_cu, occ);
  // every workgroup holds a trajectory's whole explicit state in device
  // memory: keep the pool within PLAIN_POOL_BYTES
  const double per_wg = (double)c->Emax * ((double)c->prec * 2.0 + 17.0) + (double)threads * c->K2 * 16.0;
  const double fit = std::max(1.0, std::floor((double)PLAIN_POOL_BYTES / per_wg));
  uint32_t grid = (uint32_t)std::min<double>((double)c->num_cu * per_cu, fit);
  grid = std::max<uint32_t>(1u, std::min<uint32_t>(grid, ntraj));
  if (pl.split) {  // the plain share: no more workgroups than 1.5 x its expected trajectories
    const double pf = 1.0 - std::pow(1.0 - c->eps, (double)c->htab.dep_off[c->T]);
    grid = std::min<uint32_t>(grid, (uint32_t)std::ceil(1.5 * pf * (double)ntraj) + 1u);
  }
  pl.pb.threads = threads;
  pl.pb.emax = (uint32_t)c->Emax;
  pl.pb.grid = grid;
  return QRAM_OK;
}

// split = false keeps a depolarizing context's pruned mode on the plain
// engine alone (the test entries, which export one trajectory's state).
qram_status make_plan(qram_ctx *c, int mode, uint32_t ntraj, Plan &pl, bool split) {
  const bool hybrid = split && c->dsplit && mode == QRAM_MODE_PRUNED;
  if (mode == QRAM_MODE_PLAIN || (c->general && !hybrid)) {
    pl = Plan{};
    pl.plain = true;
    return plain_plan(c, mode, ntraj, pl);
  }
  const int spt_target = c->spt[mode] ? c->spt[mode] : 16;
  std::vector<uint32_t> ems;
  if (mode == 0) {
    ems.push_back((uint32_t)c->Emax);
  } else {
    for (uint32_t addrs = 64; ems.empty() || ems.back() < (uint32_t)c->Emax; addrs *= 4)
      ems.push_back(std::min<uint32_t>((uint32_t)c->Emax, addrs * (uint32_t)c->K2));
    while ((int)ems.size() > MAXB) ems.erase(ems.begin());
  }
  pl = Plan{};
  pl.nb = (int)ems.size();
  // decode every candidate of a trajectory into shared memory when the
  // candidate buffer is small; otherwise one slice at a time
  const uint32_t ccap = cand_capacity(c);
  pl.cdec_all = ccap <= 4096u;
  pl.cdec_cap = pl.cdec_all ? ccap : (uint32_t)NCS;
  pl.persistent = (c->schedule[mode] & 1) != 0;
  const bool state_global = (c->schedule[mode] & 2) != 0;
  for (int i = 0; i < pl.nb; ++i) {
    BucketShape &b = pl.b[i];
    b.emax = ems[i];
    const uint32_t addrs = b.emax / (uint32_t)c->K2;
    const uint32_t tmax = (uint32_t)EVOLVE_MAX_THREADS[c->enc];
    uint32_t thr = pow2ceil((b.emax + spt_target - 1) / spt_target);
    thr = std::max<uint32_t>(64u, std::min<uint32_t>(tmax, thr));
    uint32_t apt = (addrs + thr - 1) / thr;
    while (apt * (uint32_t)c->K2 > (uint32_t)MAXSPT && thr < tmax) {
      thr *= 2;
      apt = (addrs + thr - 1) / thr;
    }
    if (apt * (uint32_t)c->K2 > (uint32_t)MAXSPT)
      return fail(c, QRAM_E_RANGE, "too many components per trajectory for one workgroup");
    b.threads = (int)thr;
    b.apt = apt;
    b.e_cap = apt * (uint32_t)c->K2 * thr;
    const uint32_t wb = walk_table_bytes(c->T, c->n, c->k);
    const uint32_t fixed = evolve_lds_bytes(c->M, c->D, b.threads, pl.cdec_cap, 0, false, wb);
    b.state_lds = !state_global && fixed + b.e_cap * 4u <= std::min<size_t>(c->lds_max, 96u * 1024u);
    b.lds = evolve_lds_bytes(c->M, c->D, b.threads, pl.cdec_cap, b.e_cap, b.state_lds, wb);
    if (b.lds > c->lds_max) return fail(c, QRAM_E_RANGE, "workgroup shared memory exceeds the device limit");
    int occ = evolve_occupancy(c->enc, b.state_lds, b.threads, b.lds);
    if (occ < 1) occ = 1;
    b.grid = std::max<uint32_t>(1u, std::min<uint32_t>((uint32_t)(c->num_cu * occ), ntraj));
    pl.pool_slots = std::max(pl.pool_slots, b.emax);
    pl.grid_max = std::max(pl.grid_max, b.grid);
    pl.ecap_max = std::max(pl.ecap_max, b.state_lds ? 0u : b.e_cap);
  }
  if (hybrid) {
    pl.split = true;
    return plain_plan(c, mode, ntraj, pl);
  }
  return QRAM_OK;
}

// Grow the per-trajectory buffers to `nb` trajectories and the per-workgroup
// buffers to the plan.
qram_status ensure_buffers(qram_ctx *c, uint32_t nb, const Plan *pl) {
  qram_status st;
  if (nb > c->batch_cap || c->cand_cap == 0) {
    c->cand_cap = cand_capacity(c);
    if ((st = dev_alloc(c, &c->cand, (size_t)nb * c->cand_cap))) return st;
    if ((st = dev_alloc(c, &c->ncand, nb))) return st;
    if ((st = dev_alloc(c, &c->nbad, nb))) return st;
    if ((st = dev_alloc(c, &c->ref, nb))) return st;
    if ((st = dev_alloc(c, &c->nexpl, nb))) return st;
    if ((st = dev_alloc(c, &c->order, nb))) return st;
    if ((st = dev_alloc(c, &c->digest, nb))) return st;
    if ((st = dev_alloc(c, &c->badbits, (size_t)nb * ((c->D + 63) / 64)))) return st;
    if ((st = dev_alloc(c, &c->xlist, (size_t)nb * c->D))) return st;
    if (c->eps > 0.0) {
      c->dep_cap = dep_capacity(c);
      if ((st = dev_alloc(c, &c->dep, (size_t)nb * c->dep_cap))) return st;
      if ((st = dev_alloc(c, &c->ndep, nb))) return st;
    }
    c->batch_cap = nb;
  }
  if (!c->counter) {
    if ((st = dev_alloc(c, &c->counter, MAXB))) return st;
    if ((st = dev_alloc(c, &c->bucket_base, MAXB + 2))) return st;
    if ((st = dev_alloc(c, &c->errw, 4))) return st;
    HIPCHK(c, hipMemset(c->errw, 0, 16));
  }
  if (!pl) return QRAM_OK;
  // the record pool serves the plain engine and the trajectory kernel (one
  // after the other in a split batch): sized for the larger
  size_t ps = 0;
  if (pl->plain || pl->split) {
    const size_t g = pl->pb.grid, E = (size_t)c->Emax;
    ps = g * E * c->prec;
    if ((st = grow(c, &c->pamp, &c->pamp_cap, g * E * 2))) return st;
    if ((st = grow(c, &c->phit, &c->phit_cap, g * E))) return st;
    if ((st = grow(c, &c->pgrp, &c->pgrp_cap, g * (size_t)pl->pb.threads * c->K2 * 2))) return st;
  }
  if (!pl->plain) {
    const size_t gs = (size_t)pl->grid_max * pl->ecap_max;
    if (gs > c->gstate_cap) {
      if ((st = dev_alloc(c, &c->gstate, gs))) return st;
      c->gstate_cap = gs;
    }
    for (int i = 0; i < pl->nb; ++i)
      ps = std::max(ps, (size_t)pl->b[i].grid * pl->b[i].emax * c->rec);
    size_t ds = 0;
    for (int i = 0; i < pl->nb; ++i) ds = std::max(ds, (size_t)pl->b[i].grid * pl->b[i].emax);
    if (ds > c->devl_cap) {
      if ((st = dev_alloc(c, &c->devl, ds))) return st;
      c->devl_cap = ds;
    }
  }
  if (ps > c->pool_cap) {
    if ((st = dev_alloc(c, &c->pool, ps))) return st;
    c->pool_cap = ps;
  }
  return QRAM_OK;
}

// Device bytes of the work buffers that batches of nb trajectories need
// under plan pl (what ensure_buffers allocates), and of the context's tables.
size_t buffers_bytes(const qram_ctx *c, uint32_t nb, const Plan &pl) {
  const size_t n = nb;
  size_t b = n * cand_capacity(c) * 4 + n * 5 * 4 + n * 8 + n * ((c->D + 63) / 64) * 8 + n * c->D * 2;
  b += n * ((size_t)dep_capacity(c) + 1) * 4;
  b += (2 * MAXB + 1 + 4) * 4;
  size_t ps = 0, ds = 0;  // pool words, list-index words
  if (pl.plain || pl.split) {
    const size_t g = pl.pb.grid, E = (size_t)c->Emax;
    ps = g * E * c->prec;
    b += g * E * (16 + 1) + g * (size_t)pl.pb.threads * c->K2 * 16;
  }
  if (!pl.plain) {
    b += (size_t)pl.grid_max * pl.ecap_max * 4;
    for (int i = 0; i < pl.nb; ++i) {
      ps = std::max(ps, (size_t)pl.b[i].grid * pl.b[i].emax * c->rec);
      ds = std::max(ds, (size_t)pl.b[i].grid * pl.b[i].emax);
    }
  }
  return b + ps * 2 + ds * 4;
}

size_t table_bytes(const qram_ctx *c) {
  return (size_t)c->D * 4 + (size_t)(c->emax + std::max(c->emax, c->prec) + 1) * 8 * 2 + sizeof(Tables) + (size_t)(MAXT + 1) * 8 +
         (size_t)2 * c->T * (97 + (1 << c->k)) * 8;
}

uint32_t batch_size(const qram_ctx *c, uint32_t ntraj);
qram_status make_plan(qram_ctx *c, int mode, uint32_t ntraj, Plan &pl, bool split = true);

uint32_t batch_size(const qram_ctx *c, uint32_t ntraj) {
  // keep the per-trajectory buffers within about 2 GiB
  const double per = (double)cand_capacity(c) * 4.0 + (double)c->D * 2.0 +
                     (double)((c->D + 63) / 64) * 8.0 + 64.0;
  double nb = (2.0 * 1024 * 1024 * 1024) / per;
  nb = std::max(256.0, std::min(nb, 262144.0));
  return std::min<uint32_t>(ntraj, (uint32_t)nb);
}

Run base_run(qram_ctx *c, int mode, uint64_t seed, const Plan *pl) {
  Run r;
  std::memset(&r, 0, sizeof(Run));  // padding too: graph replay compares runs bytewise
  r.seed = seed;
  r.mode = mode;
  r.cand_cap = c->cand_cap;
  r.tier2_slow = c->tier2_global ? 1u : 0u;
  if (pl) r.cdec_all = pl->cdec_all ? 1u : 0u;
  if (pl) {
    r.nbkt = (uint32_t)pl->nb;
    for (int i = 0; i < pl->nb; ++i) r.bkt_emax[i] = pl->b[i].emax;
    r.pool_slots = pl->pool_slots;
    r.persistent = pl->persistent ? 1u : 0u;
  }
  r.cand = c->cand;
  r.ncand = c->ncand;
  r.digest = c->digest;
  r.badbits = c->badbits;
  r.nbad = c->nbad;
  r.ref = c->ref;
  r.xlist = c->xlist;
  r.nexpl = c->nexpl;
  r.order = c->order;
  r.bucket_base = c->bucket_base;
  r.counter = c->counter;
  r.gstate = c->gstate;
  r.pool = c->pool;
  r.devl = c->devl;
  r.err = c->errw;
  if (c->eps > 0.0) {
    r.dep = c->dep;
    r.ndep = c->ndep;
    r.dep_cap = c->dep_cap;
  }
  r.prec = (uint32_t)c->prec;
  if (pl) r.pslab = pl->pslab;
  if (pl) r.dsplit = pl->split ? 1u : 0u;
  r.pamp = c->pamp;
  r.phit = c->phit;
  r.pgrp = c->pgrp;
  return r;
}

uint32_t sample_grid(const qram_ctx *c, uint32_t ntraj) {
  return std::max<uint32_t>(1u, std::min<uint32_t>(ntraj, (uint32_t)c->num_cu * 8u));
}

constexpr size_t EVB = 4 + 2 * MAXB;  // timing events per batch

// be (optional): two events per bucket, recorded around its launch.
qram_status launch_buckets(qram_ctx *c, const Plan &pl, Run r, hipStream_t s, hipEvent_t *be = nullptr) {
  for (int i = 0; i < pl.nb; ++i) {
    const BucketShape &b = pl.b[i];
    r.bucket = (uint32_t)i;
    r.apt = b.apt;
    r.e_cap = b.e_cap;
    r.pool_slots = b.emax;  // a workgroup's records: one per explicit component of the bucket
    if (be) HIPCHK(c, hipEventRecord(be[2 * i], s));
    HIPCHK(c, launch_evolve(c->dtab, r, c->enc, b.grid, b.threads, b.lds, b.state_lds, s));
    if (be) HIPCHK(c, hipEventRecord(be[2 * i + 1], s));
  }
  return QRAM_OK;
}

// Enqueue sampling (unless forced), classification, bucketing and evolution
// of one batch on stream s.  With `timed`, events bracket the three stages.
qram_status enqueue_batch(qram_ctx *c, const Plan &pl, Run r, hipStream_t s,
                          bool timed, bool skip_sample, bool capture = false) {
  const uint32_t nt = r.ntraj;
  hipEvent_t e[4] = {c->ev[0], c->ev[1], c->ev[2], c->ev[3]};
  if (capture) timed = false;
  hipEvent_t *be = nullptr;
  if (!timed && !capture && c->timing) {  // async stage timing: pooled events
    while (c->tev.size() < c->tev_used + EVB) {
      hipEvent_t x;
      HIPCHK(c, hipEventCreate(&x));
      c->tev.push_back(x);
    }
    for (int i = 0; i < 4; ++i) e[i] = c->tev[c->tev_used + i];
    be = &c->tev[c->tev_used + 4];
    c->tev_used += EVB;
    c->tev_launches += (uint32_t)pl.nb;
    c->tev_nb.push_back(pl.nb);
    for (int i = 0; i < MAXB; ++i) c->tev_emax[i] = i < pl.nb ? pl.b[i].emax : 0u;
    timed = true;
  }
  if (timed) HIPCHK(c, hipEventRecord(e[0], s));
  if (!skip_sample) HIPCHK(c, launch_sample(c->dtab, r, nt, sample_grid(c, nt), s));
  if (r.dep) HIPCHK(c, launch_sample_depol(c->dtab, r, sample_grid(c, nt), s));
  if (timed) HIPCHK(c, hipEventRecord(e[1], s));
  HIPCHK(c, launch_classify(c->dtab, r, nt, sample_grid(c, nt), c->D, c->mark_subtree, s));
  if (!pl.plain) HIPCHK(c, launch_order(c->dtab, r, s));
  if (timed) HIPCHK(c, hipEventRecord(e[2], s));
  if (pl.plain) {
    HIPCHK(c, launch_plain(c->dtab, r, c->enc, pl.pvar, pl.pb.grid, pl.pb.threads, pl.plds, s));
    c->plain_used_thr[r.mode] = pl.pb.threads;
  } else {
    qram_status st = launch_buckets(c, pl, r, s, be);
    if (st) return st;
    if (pl.split) {  // the trajectories that drew a depolarizing fault
      HIPCHK(c, launch_plain(c->dtab, r, c->enc, pl.pvar, pl.pb.grid, pl.pb.threads, pl.plds, s));
      c->plain_used_thr[QRAM_MODE_PRUNED] = pl.pb.threads;
    }
  }
  if (timed) HIPCHK(c, hipEventRecord(e[3], s));
  return QRAM_OK;
}

// The batch as one graph: captured on the context's stream, instantiated
// once (or updated in place when the executable graph exists) and launched
// on stream s.  The captured work holds no memset node.
// FNV-1a over the launch shapes of a plan (what a captured graph bakes in
// besides the kernel arguments).
uint64_t plan_signature(const Plan &pl) {
  uint64_t h = 0xcbf29ce484222325ull;
  auto mix = [&h](uint64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (v >> (8 * i)) & 0xFFu;
      h *= 0x100000001b3ull;
    }
  };
  mix((uint64_t)pl.nb);
  mix(pl.plain ? 1u : 0u);
  mix(pl.split ? 1u : 0u);
  mix(pl.plds);
  mix(pl.pslab);
  mix((uint64_t)pl.pb.threads);
  mix(pl.pb.grid);
  mix((uint64_t)pl.pvar);
  for (int i = 0; i < pl.nb; ++i) {
    const BucketShape &b = pl.b[i];
    mix(b.emax);
    mix((uint64_t)b.threads);
    mix(b.apt);
    mix(b.e_cap);
    mix(b.state_lds ? 1u : 0u);
    mix(b.lds);
    mix(b.grid);
  }
  return h;
}

qram_status launch_batch_graph(qram_ctx *c, const Plan &pl, const Run &r,
                               hipStream_t s) {
  const uint64_t sig = plan_signature(pl);
  if (c->gexec && sig == c->graph_sig && std::memcmp(&r, &c->graph_run, sizeof(Run)) == 0) {
    HIPCHK(c, hipGraphLaunch(c->gexec, s));  // same work as captured: replay
    return QRAM_OK;
  }
  hipGraph_t g = nullptr;
  HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  qram_status st = enqueue_batch(c, pl, r, c->stream, false, false, true);
  const hipError_t ec = hipStreamEndCapture(c->stream, &g);
  if (st) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  HIPCHK(c, ec);
  bool ok = false;
  if (c->gexec) {
    hipGraphNode_t bad = nullptr;
    hipGraphExecUpdateResult res;
    ok = hipGraphExecUpdate(c->gexec, g, &bad, &res) == hipSuccess && res == hipGraphExecUpdateSuccess;
    if (!ok) {
      (void)hipGetLastError();
      (void)hipGraphExecDestroy(c->gexec);
      c->gexec = nullptr;
    }
  }
  if (!ok) {
    const hipError_t ei = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      c->gexec = nullptr;
      (void)hipGraphDestroy(g);
      HIPCHK(c, ei);
    }
  }
  (void)hipGraphDestroy(g);
  c->graph_run = r;
  c->graph_sig = sig;
  HIPCHK(c, hipGraphLaunch(c->gexec, s));
  return QRAM_OK;
}

qram_status check_err(qram_ctx *c) {
  uint32_t e = 0;
  HIPCHK(c, hipMemcpy(&e, c->errw, 4, hipMemcpyDeviceToHost));
  if (e) {
    HIPCHK(c, hipMemset(c->errw, 0, 4));
    if (e & ERR_CAND) return fail(c, QRAM_E_CAPACITY, "candidate buffer overflow");
    if (e & ERR_LIST) return fail(c, QRAM_E_CAPACITY, "explicit site list overflow");
    if (e & ERR_DEP) return fail(c, QRAM_E_CAPACITY, "depolarizing fault buffer overflow");
  }
  return QRAM_OK;
}

qram_status check_args(qram_ctx *c, uint64_t traj0, uint32_t ntraj) {
  if (!c) return fail(nullptr, QRAM_E_INVAL, "null context");
  if (traj0 + (uint64_t)ntraj > (1ull << 32))
    return fail(c, QRAM_E_RANGE, "traj0 + ntraj exceeds 2^32");
  HIPCHK(c, hipSetDevice(c->device));
  return QRAM_OK;
}

qram_status ensure_out(qram_ctx *c, uint32_t nb) {
  if (nb > c->out_cap) {
    qram_status st;
    if ((st = dev_alloc(c, &c->fid_tmp, nb))) return st;
    if ((st = dev_alloc(c, &c->st_tmp, nb))) return st;
    c->out_cap = nb;
  }
  return QRAM_OK;
}

// Runs trajectories [traj0, traj0+ntraj) in batches.  Outputs go to device
// arrays d_fid/d_st (async) or through the context's staging buffers to host
// arrays h_fid/h_st (sync).
qram_status run_mode(qram_ctx *c, int mode, uint64_t seed, uint64_t traj0,
                     uint32_t ntraj, double *d_fid, qram_traj_stats *d_st,
                     double *h_fid, qram_traj_stats *h_st, hipStream_t s,
                     bool sync, uint32_t *h_jlog = nullptr, uint32_t jcap = 0,
                     uint32_t *h_njl = nullptr) {
  qram_status st = check_args(c, traj0, ntraj);
  if (st) return st;
  if (ntraj == 0) return QRAM_OK;
  const uint32_t nb = batch_size(c, ntraj);
  Plan pl;
  if ((st = make_plan(c, mode, nb, pl))) return st;
  if ((st = ensure_buffers(c, nb, &pl))) return st;
  if (sync && (st = ensure_out(c, nb))) return st;
  const bool logs = sync && h_njl != nullptr;
  if (logs) {
    if ((st = grow(c, &c->djlog, &c->djlog_cap, (size_t)nb * std::max<uint32_t>(jcap, 1u)))) return st;
    if ((st = grow(c, &c->djn, &c->djn_cap, (size_t)nb))) return st;
  }
  const bool timed = sync && ntraj <= nb;
  for (uint32_t b0 = 0; b0 < ntraj; b0 += nb) {
    const uint32_t cnt = std::min(nb, ntraj - b0);
    Run r = base_run(c, mode, seed, &pl);
    r.traj0 = (uint32_t)(traj0 + b0);
    r.ntraj = cnt;
    r.fid = sync ? c->fid_tmp : d_fid + b0;
    r.st = sync ? (h_st ? c->st_tmp : nullptr) : (d_st ? d_st + b0 : nullptr);
    if (logs) {
      r.jlog = c->djlog;
      r.jn = c->djn;
      r.jcap = jcap;
    }
    if (c->use_graph) {
      if (timed) HIPCHK(c, hipEventRecord(c->ev[0], s));
      if ((st = launch_batch_graph(c, pl, r, s))) return st;
      if (timed) HIPCHK(c, hipEventRecord(c->ev[3], s));
    } else if ((st = enqueue_batch(c, pl, r, s, timed, false))) {
      return st;
    }
    if (sync) {
      HIPCHK(c, hipMemcpyAsync(h_fid + b0, c->fid_tmp, cnt * sizeof(double), hipMemcpyDeviceToHost, s));
      if (h_st)
        HIPCHK(c, hipMemcpyAsync(h_st + b0, c->st_tmp, cnt * sizeof(qram_traj_stats), hipMemcpyDeviceToHost, s));
      if (logs) {
        HIPCHK(c, hipMemcpyAsync(h_njl + b0, c->djn, cnt * 4, hipMemcpyDeviceToHost, s));
        if (jcap && h_jlog)
          HIPCHK(c, hipMemcpyAsync(h_jlog + (size_t)b0 * jcap, c->djlog, (size_t)cnt * jcap * 4,
                                   hipMemcpyDeviceToHost, s));
      }
      HIPCHK(c, hipStreamSynchronize(s));
    }
  }
  if (sync) {
    if (timed && c->use_graph) {  // one graph: the whole batch counts as evolution
      float ms;
      HIPCHK(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[3]));
      c->last_ms[0] = c->last_ms[1] = 0.0;
      c->last_ms[2] = ms;
    } else if (timed) {
      float ms;
      for (int i = 0; i < 3; ++i) {
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
        c->last_ms[i] = ms;
      }
    }
    return check_err(c);
  }
  return QRAM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

qram_status qram_create(int n_addr, int k_data, qram_encoding enc, double gamma,
                        const uint32_t *memory_bits, qram_ctx **out) {
  qram_params p{};
  p.n_addr = n_addr;
  p.k_data = k_data;
  p.enc = enc;
  p.gamma = gamma;
  p.eps = 0.0;
  p.memory_bits = memory_bits;
  return qram_create_ex(&p, out);
}

qram_status qram_create_ex(const qram_params *p, qram_ctx **out) {
  if (!out || !p || !p->memory_bits) return fail(nullptr, QRAM_E_INVAL, "null argument");
  *out = nullptr;
  const int n_addr = p->n_addr, k_data = p->k_data;
  const qram_encoding enc = p->enc;
  const double gamma = p->gamma, eps = p->eps;
  const uint32_t *memory_bits = p->memory_bits;
  if (enc != QRAM_QUBIT && enc != QRAM_QUTRIT) return fail(nullptr, QRAM_E_INVAL, "unknown encoding");
  if (!(gamma >= 0.0 && gamma < 1.0)) return fail(nullptr, QRAM_E_INVAL, "gamma must lie in [0, 1)");
  if (!(eps >= 0.0 && eps < 1.0)) return fail(nullptr, QRAM_E_INVAL, "eps must lie in [0, 1)");
  const int nmax = enc == QRAM_QUTRIT ? 14 : 15;
  if (n_addr < 1 || n_addr > nmax) return fail(nullptr, QRAM_E_RANGE, "n_addr out of range");
  if (k_data < 1 || k_data > 8 || k_data > n_addr) return fail(nullptr, QRAM_E_RANGE, "k_data out of range (1..8, k <= n)");
  if (enc == QRAM_QUBIT && n_addr + k_data > 16)
    return fail(nullptr, QRAM_E_RANGE, "qubit encoding needs n + k <= 16 (at most 65536 components)");
  std::vector<double> cin;
  if (p->input_amp) {  // normalised general input
    double norm = 0.0;
    cin.assign(p->input_amp, p->input_amp + 2 * ((size_t)1 << n_addr));
    for (double v : cin) norm += v * v;
    if (!(norm > 0.0) || !std::isfinite(norm)) return fail(nullptr, QRAM_E_INVAL, "input amplitudes must be finite and not all zero");
    const double f = 1.0 / std::sqrt(norm);
    for (double &v : cin) v *= f;
  }
  std::vector<double> cab;  // normalised c_ij of every (address, bus word) pair
  if (p->input_ab) {
    if (p->input_amp || p->input_bus) return fail(nullptr, QRAM_E_INVAL, "input_ab excludes input_amp and input_bus");
    double norm = 0.0;
    cab.assign(p->input_ab, p->input_ab + 2 * (((size_t)1 << n_addr) << k_data));
    for (double v : cab) norm += v * v;
    if (!(norm > 0.0) || !std::isfinite(norm)) return fail(nullptr, QRAM_E_INVAL, "input amplitudes must be finite and not all zero");
    const double f = 1.0 / std::sqrt(norm);
    for (double &v : cab) v *= f;
  }
  if (p->truncate && (p->w_max < 0 || p->w_max > k_data)) return fail(nullptr, QRAM_E_INVAL, "w_max must lie in 0..k");
  qram_ctx *c = new (std::nothrow) qram_ctx();
  if (!c) return fail(nullptr, QRAM_E_NOMEM, "host allocation failed");
  c->n = n_addr;
  c->k = k_data;
  c->enc = enc == QRAM_QUBIT ? QUBIT : QUTRIT;
  c->gamma = gamma;
  c->eps = eps;
  // the trajectory kernel covers damping on the data-loading input with up
  // to six qubit data bits; everything else runs on the plain engine
  c->general = eps > 0.0 || p->input_amp || p->input_bus || p->input_ab || p->truncate ||
               (c->enc == QUBIT && k_data > 6);
  // a trajectory that drew no depolarizing fault is a damping-only one: on
  // the data-loading input the trajectory kernel runs it
  c->dsplit = eps > 0.0 && !p->input_amp && !p->input_bus && !p->input_ab && !p->truncate &&
              !(c->enc == QUBIT && k_data > 6);
  c->T = 6 * n_addr + 2 * k_data;
  c->M = 2 * ((1 << n_addr) - 1);
  c->D = 1 << n_addr;
  // qubit: one component per (address, bus word after the wall); qutrit: one
  // per address, or per (address, bus word) pair with a pair input
  c->K2 = (c->enc == QUBIT || !cab.empty()) ? (1 << k_data) : 1;
  c->Emax = c->D * c->K2;
  // excitations per component: the CNOT copies are the only gates that
  // create them in the qubit circuit (<= 2n, plus k bus bits); the qutrit
  // circuit adds at most one router per store/unstore and one per fetch
  c->lmax = c->enc == QUBIT ? 2 * n_addr + k_data : 4 * n_addr + k_data;
  c->emax = (c->T - 1) * c->lmax;
  // record: count, bus word, lmax sites (+ the data tokens' sites and the
  // split set of a shared qubit list)
  c->rec = (c->lmax + 2 + (c->enc == QUBIT ? k_data + 1 : 0) + 1) & ~1;
  // plain-engine record: count, bus word, exposure, phase, sites (16-byte records)
  c->prec = (c->lmax + PLAIN_EXTRA + 4 + 7) & ~7;
  const double lw = c->emax * std::log(1.0 - gamma);
  if (lw < -690.0) {
    delete c;
    return fail(nullptr, QRAM_E_RANGE, "gamma too large: damping weights underflow double precision");
  }
  c->mem.assign(memory_bits, memory_bits + c->D);
  for (auto &m : c->mem) m &= (1u << k_data) - 1u;
  {  // the input's (address, bus word) pairs with their normalised amplitudes
    const uint32_t K = 1u << k_data;
    for (uint32_t i = 0; i < (uint32_t)c->D; ++i) {
      if (!cab.empty()) {
        for (uint32_t j = 0; j < K; ++j) {
          const double re = cab[2 * ((size_t)i * K + j)], im = cab[2 * ((size_t)i * K + j) + 1];
          if (re == 0.0 && im == 0.0) continue;
          c->in_idx.push_back(i << 8 | j);
          c->in_amp.push_back(re);
          c->in_amp.push_back(im);
        }
        continue;
      }
      const double re = cin.empty() ? 1.0 / std::sqrt((double)c->D) : cin[2 * i];
      const double im = cin.empty() ? 0.0 : cin[2 * i + 1];
      if (re == 0.0 && im == 0.0) continue;
      const uint32_t j = p->input_bus ? (p->input_bus[i] & (K - 1u)) : 0u;
      c->in_idx.push_back(i << 8 | j);
      c->in_amp.push_back(re);
      c->in_amp.push_back(im);
    }
  }
  std::string why;
  if (!build_tables(c, why)) {
    delete c;
    return fail(nullptr, QRAM_E_INVAL, "schedule: " + why);
  }  // plain engine records: an X-type depolarizing fault on an idle site adds
  // one excitation to every branch (a stray), so the lists hold up to the
  // trajectory's fault capacity beyond lmax
  if (c->eps > 0.0)
    c->prec = (int)((std::min<uint32_t>((uint32_t)(c->lmax + PLAIN_EXTRA) + dep_capacity(c), (uint32_t)(c->M + c->lmax)) +
                     4u + 7u) & ~7u);

  auto bail = [&](qram_status st) {
    std::string m = c->err;
    qram_destroy(c);
    return fail(nullptr, st, m);
  };
  if (hipGetDevice(&c->device) != hipSuccess) return bail(fail(c, QRAM_E_DEVICE, "no HIP device"));
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) return bail(fail(c, QRAM_E_DEVICE, "hipGetDeviceProperties failed"));
  c->num_cu = prop.multiProcessorCount;
  c->scratch = scratch_address(c->device);
  int dyn = 0;
  if (evolve_prepare((int)prop.sharedMemPerBlock, &dyn) == hipSuccess) {
    c->lds_max = (size_t)dyn;  // dynamic shared memory an evolution launch may take
  } else {
    (void)hipGetLastError();
    c->lds_max = std::min<size_t>(prop.sharedMemPerBlock, 64 * 1024) - 1024;
  }
  if (plain_prepare((int)prop.sharedMemPerBlock) != hipSuccess) (void)hipGetLastError();  // (large workgroups then fit less)
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) return bail(fail(c, QRAM_E_DEVICE, "stream creation failed"));
  for (auto &e : c->ev)
    if (hipEventCreate(&e) != hipSuccess) return bail(fail(c, QRAM_E_DEVICE, "event creation failed"));
  qram_status st;
  if ((st = dev_alloc(c, &c->dmem, c->D))) return bail(st);
  // exponents -emax .. phi: phi covers a plain-engine list's length too,
  // which with depolarizing strays can exceed emax
  const int phi = std::max(c->emax, c->prec);
  std::vector<double> wp(c->emax + phi + 1), ap(c->emax + phi + 1);
  const double a = std::sqrt(1.0 - gamma);
  for (int m = 0; m <= c->emax + phi; ++m) {
    wp[m] = std::pow(1.0 - gamma, (double)(m - c->emax));
    ap[m] = std::pow(a, (double)(m - c->emax));
  }
  if ((st = dev_alloc(c, &c->dwpow, wp.size()))) return bail(st);
  if ((st = dev_alloc(c, &c->dapow, ap.size()))) return bail(st);
  if ((st = dev_alloc(c, &c->dtab, 1))) return bail(st);
  // per-slice factor tables: exposure through slice s of each 5-bit chunk
  // of the address bits, of each data-token set, and of the routers
  const int nd = 1 << c->k, nfs = 96 + nd + 1;
  std::vector<double> ft((size_t)2 * c->T * nfs);
  for (int which = 0; which < 2; ++which) {
    const std::vector<double> &pw = which ? ap : wp;
    for (int sl = 0; sl < c->T; ++sl) {
      double *row = ft.data() + ((size_t)which * c->T + sl) * nfs;
      for (int x = 0; x < 96; ++x) {
        const int ch = x >> 5, v = x & 31;
        int e = 0;
        for (int b = 0; b < 5; ++b) {
          const int pbit = 5 * ch + b;
          if (pbit < c->n && ((v >> b) & 1)) e += c->htab.cntA[sl][c->n - 1 - pbit];
        }
        row[x] = pw[c->emax + e];
      }
      for (int v = 0; v < nd; ++v) {
        int e = 0;
        for (int b = 0; b < c->k; ++b)
          if ((v >> b) & 1) e += c->htab.cntD[sl][b];
        row[96 + v] = pw[c->emax + e];
      }
      row[96 + nd] = pw[c->emax + c->htab.cntR[sl]];
    }
  }
  // no-jump sums over all addresses (every branch on its no-jump orbit):
  // the total weight through each slice, and the final overlap and weight
  std::vector<double> ctot(c->T);
  auto nojump_sum = [&](int which, int sl) {
    const double *row = ft.data() + ((size_t)which * c->T + sl) * nfs;
    double sum = 0.0, comp = 0.0;  // Neumaier
    for (int a = 0; a < c->D; ++a) {
      double g = 0.0;
      if (c->enc == QUBIT)
        for (int b = 0; b < nd; ++b) g += row[96 + b];
      else
        g = row[96 + (c->mem[a] & (uint32_t)(nd - 1))];
      const double x = row[a & 31] * row[32 + ((a >> 5) & 31)] * row[64 + ((a >> 10) & 31)] * row[96 + nd] * g;
      const double t = sum + x;
      comp += std::fabs(sum) >= std::fabs(x) ? (sum - t) + x : (x - t) + sum;
      sum = t;
    }
    return sum + comp;
  };
  for (int sl = 0; sl < c->T; ++sl) ctot[sl] = nojump_sum(0, sl);
  c->htab.w_nojump = ctot[c->T - 1];
  c->htab.ov_nojump = nojump_sum(1, c->T - 1);
  if ((st = dev_alloc(c, &c->dctot, ctot.size()))) return bail(st);
  if ((st = dev_alloc(c, &c->dftab, ft.size()))) return bail(st);
  if (!cin.empty()) {
    if ((st = dev_alloc(c, &c->dcin, cin.size()))) return bail(st);
    if (hipMemcpy(c->dcin, cin.data(), cin.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
      return bail(fail(c, QRAM_E_DEVICE, "input upload failed"));
    c->htab.cin = c->dcin;
  }
  if (p->input_bus) {
    std::vector<uint32_t> jin(p->input_bus, p->input_bus + c->D);
    for (auto &j : jin) j &= (1u << k_data) - 1u;
    if ((st = dev_alloc(c, &c->djin, jin.size()))) return bail(st);
    if (hipMemcpy(c->djin, jin.data(), jin.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
      return bail(fail(c, QRAM_E_DEVICE, "input upload failed"));
    c->htab.jin = c->djin;
  }
  c->htab.trunc_w = (p->truncate && p->w_max < k_data) ? p->w_max : -1;
  if (!cab.empty()) {
    // per address: presence, one bus word (its amplitude and word go to
    // cin/jin); per component: the amplitude after the first wall
    const int K = 1 << k_data;
    std::vector<double> cs(2 * (size_t)c->D, 0.0);
    std::vector<uint32_t> js(c->D, 0u);
    std::vector<uint8_t> af(c->D, 0);
    for (int i = 0; i < c->D; ++i) {
      int m = 0, jl = 0;
      for (int j = 0; j < K; ++j) {
        const size_t x = (size_t)i * K + j;
        if (cab[2 * x] != 0.0 || cab[2 * x + 1] != 0.0) {
          ++m;
          jl = j;
        }
      }
      af[i] = (uint8_t)((m > 0 ? 1 : 0) | (m == 1 ? 2 : 0));
      if (m == 1) {
        cs[2 * i] = cab[2 * ((size_t)i * K + jl)];
        cs[2 * i + 1] = cab[2 * ((size_t)i * K + jl) + 1];
        js[i] = (uint32_t)jl;
      }
      if (m > 1 && c->htab.trunc_w >= 0) return bail(fail(c, QRAM_E_INVAL, "truncation needs one bus word per address"));
    }
    std::vector<double> ca(2 * (size_t)c->D * c->K2);
    if (c->enc == QUBIT) {  // 2^(-k/2) sum_j c_ij (-1)^(beta . j), j ascending
      const double h = 1.0 / std::sqrt((double)K);
      for (int i = 0; i < c->D; ++i)
        for (int b = 0; b < K; ++b) {
          double re = 0.0, im = 0.0;
          for (int j = 0; j < K; ++j) {
            const size_t x = (size_t)i * K + j;
            const bool neg = __builtin_popcount((unsigned)(b & j)) & 1;
            re += neg ? -cab[2 * x] : cab[2 * x];
            im += neg ? -cab[2 * x + 1] : cab[2 * x + 1];
          }
          ca[2 * ((size_t)i * K + b)] = re * h;
          ca[2 * ((size_t)i * K + b) + 1] = im * h;
        }
    } else {
      ca = cab;
    }
    if ((st = dev_alloc(c, &c->dcab, cab.size())) || (st = dev_alloc(c, &c->dcamp, ca.size())) ||
        (st = dev_alloc(c, &c->daflag, af.size())) || (st = dev_alloc(c, &c->dcin, cs.size())) ||
        (st = dev_alloc(c, &c->djin, js.size())))
      return bail(st);
    if (hipMemcpy(c->dcab, cab.data(), cab.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->dcamp, ca.data(), ca.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->daflag, af.data(), af.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->dcin, cs.data(), cs.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->djin, js.data(), js.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
      return bail(fail(c, QRAM_E_DEVICE, "input upload failed"));
    c->htab.cab = c->dcab;
    c->htab.camp = c->dcamp;
    c->htab.aflag = c->daflag;
    c->htab.cin = c->dcin;
    c->htab.jin = c->djin;
  }
  c->htab.mem = c->dmem;
  c->htab.wpow = c->dwpow;
  c->htab.apow = c->dapow;
  c->htab.ftab_w = c->dftab;
  c->htab.ftab_a = c->dftab + (size_t)c->T * nfs;
  c->htab.nfs = nfs;
  c->htab.ctot = c->dctot;
  if (hipMemcpy(c->dmem, c->mem.data(), c->D * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->dwpow, wp.data(), wp.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->dapow, ap.data(), ap.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->dftab, ft.data(), ft.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->dctot, ctot.data(), ctot.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->dtab, &c->htab, sizeof(Tables), hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(c, QRAM_E_DEVICE, "table upload failed"));
  *out = c;
  return QRAM_OK;
}

void qram_destroy(qram_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  dev_free(&c->dtab);
  dev_free(&c->dmem);
  dev_free(&c->dwpow);
  dev_free(&c->dapow);
  dev_free(&c->dftab);
  dev_free(&c->dctot);
  dev_free(&c->cand);
  dev_free(&c->ncand);
  dev_free(&c->nbad);
  dev_free(&c->ref);
  dev_free(&c->nexpl);
  dev_free(&c->order);
  dev_free(&c->counter);
  dev_free(&c->bucket_base);
  dev_free(&c->errw);
  dev_free(&c->badbits);
  dev_free(&c->digest);
  dev_free(&c->xlist);
  dev_free(&c->pool);
  dev_free(&c->devl);
  dev_free(&c->gstate);
  dev_free(&c->fid_tmp);
  dev_free(&c->st_tmp);
  dev_free(&c->uaux);
  dev_free(&c->dcin);
  dev_free(&c->djin);
  dev_free(&c->dcab);
  dev_free(&c->dcamp);
  dev_free(&c->daflag);
  dev_free(&c->dep);
  dev_free(&c->ndep);
  dev_free(&c->dexp);
  dev_free(&c->dexpamp);
  dev_free(&c->pamp);
  dev_free(&c->pgrp);
  dev_free(&c->phit);
  dev_free(&c->djlog);
  dev_free(&c->djn);
  for (auto &e : c->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto &e : c->tev) (void)hipEventDestroy(e);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char *qram_last_error(const qram_ctx *c) {
  return c ? c->err.c_str() : g_create_error.c_str();
}

qram_status qram_sample_faults(qram_ctx *c, uint64_t seed, uint64_t traj0,
                               uint32_t ntraj, uint32_t *n_cand,
                               uint64_t *cand_digest, uint32_t *n_bad,
                               uint64_t *bad_bits, uint32_t *cand_L,
                               uint64_t cand_cap) {
  qram_status st = check_args(c, traj0, ntraj);
  if (st) return st;
  if (!n_cand) return fail(c, QRAM_E_INVAL, "n_cand is required");
  if (ntraj == 0) return QRAM_OK;
  const uint32_t nb = batch_size(c, ntraj);
  if ((st = ensure_buffers(c, nb, nullptr))) return st;
  const int w64 = (c->D + 63) / 64;
  uint64_t written = 0;
  bool overflow = false;
  std::vector<uint32_t> hc;
  for (uint32_t b0 = 0; b0 < ntraj; b0 += nb) {
    const uint32_t cnt = std::min(nb, ntraj - b0);
    Run r = base_run(c, 0, seed, nullptr);
    r.traj0 = (uint32_t)(traj0 + b0);
    r.ntraj = cnt;
    HIPCHK(c, launch_sample(c->dtab, r, cnt, sample_grid(c, cnt), c->stream));
    if (r.dep) HIPCHK(c, launch_sample_depol(c->dtab, r, sample_grid(c, cnt), c->stream));
    HIPCHK(c, launch_classify(c->dtab, r, cnt, sample_grid(c, cnt), c->D, c->mark_subtree, c->stream));
    HIPCHK(c, launch_digest(r, cnt, c->stream));
    HIPCHK(c, hipMemcpyAsync(n_cand + b0, c->ncand, cnt * 4, hipMemcpyDeviceToHost, c->stream));
    if (cand_digest) HIPCHK(c, hipMemcpyAsync(cand_digest + b0, c->digest, cnt * 8, hipMemcpyDeviceToHost, c->stream));
    if (n_bad) HIPCHK(c, hipMemcpyAsync(n_bad + b0, c->nbad, cnt * 4, hipMemcpyDeviceToHost, c->stream));
    if (bad_bits)
      HIPCHK(c, hipMemcpyAsync(bad_bits + (size_t)b0 * w64, c->badbits, (size_t)cnt * w64 * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (cand_L && !overflow) {
      uint64_t need = written;
      for (uint32_t t = 0; t < cnt; ++t) need += std::min(n_cand[b0 + t], c->cand_cap);
      if (need > cand_cap) {
        overflow = true;
      } else {
        hc.resize((size_t)cnt * c->cand_cap);
        HIPCHK(c, hipMemcpy(hc.data(), c->cand, hc.size() * 4, hipMemcpyDeviceToHost));
        for (uint32_t t = 0; t < cnt; ++t) {
          const uint32_t m = std::min(n_cand[b0 + t], c->cand_cap);
          std::memcpy(cand_L + written, hc.data() + (size_t)t * c->cand_cap, m * 4);
          written += m;
        }
      }
    }
  }
  if ((st = check_err(c))) return st;
  if (overflow) return fail(c, QRAM_E_CAPACITY, "cand_L too small for the candidate dump");
  return QRAM_OK;
}

qram_status qram_sample_depol(qram_ctx *c, uint64_t seed, uint64_t traj0, uint32_t ntraj,
                              uint32_t *n_dep, uint32_t *dep, uint64_t cap) {
  qram_status st = check_args(c, traj0, ntraj);
  if (st) return st;
  if (!n_dep) return fail(c, QRAM_E_INVAL, "n_dep is required");
  if (c->eps <= 0.0) {
    std::memset(n_dep, 0, (size_t)ntraj * 4);
    return QRAM_OK;
  }
  if (ntraj == 0) return QRAM_OK;
  const uint32_t nb = batch_size(c, ntraj);
  if ((st = ensure_buffers(c, nb, nullptr))) return st;
  uint64_t written = 0;
  bool overflow = false;
  std::vector<uint32_t> hd;
  for (uint32_t b0 = 0; b0 < ntraj; b0 += nb) {
    const uint32_t cnt = std::min(nb, ntraj - b0);
    Run r = base_run(c, 0, seed, nullptr);
    r.traj0 = (uint32_t)(traj0 + b0);
    r.ntraj = cnt;
    HIPCHK(c, launch_sample_depol(c->dtab, r, sample_grid(c, cnt), c->stream));
    HIPCHK(c, hipMemcpyAsync(n_dep + b0, c->ndep, cnt * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (dep && !overflow) {
      uint64_t need = written;
      for (uint32_t t = 0; t < cnt; ++t) need += std::min(n_dep[b0 + t], c->dep_cap);
      if (need > cap) {
        overflow = true;
      } else {
        hd.resize((size_t)cnt * c->dep_cap);
        HIPCHK(c, hipMemcpy(hd.data(), c->dep, hd.size() * 4, hipMemcpyDeviceToHost));
        for (uint32_t t = 0; t < cnt; ++t) {
          const uint32_t m = std::min(n_dep[b0 + t], c->dep_cap);
          std::memcpy(dep + written, hd.data() + (size_t)t * c->dep_cap, m * 4);
          written += m;
        }
      }
    }
  }
  if ((st = check_err(c))) return st;
  if (overflow) return fail(c, QRAM_E_CAPACITY, "dep buffer too small for the dump");
  return QRAM_OK;
}

qram_status qram_run_full(qram_ctx *c, uint64_t seed, uint64_t traj0,
                          uint32_t ntraj, double *fid, qram_traj_stats *st) {
  if (!fid) return fail(c, QRAM_E_INVAL, "fid is required");
  return run_mode(c, 0, seed, traj0, ntraj, nullptr, nullptr, fid, st, c ? c->stream : nullptr, true);
}

qram_status qram_run_pruned(qram_ctx *c, uint64_t seed, uint64_t traj0,
                            uint32_t ntraj, double *fid, qram_traj_stats *st) {
  if (!fid) return fail(c, QRAM_E_INVAL, "fid is required");
  return run_mode(c, 1, seed, traj0, ntraj, nullptr, nullptr, fid, st, c ? c->stream : nullptr, true);
}

qram_status qram_run_full_async(qram_ctx *c, uint64_t seed, uint64_t traj0,
                                uint32_t ntraj, double *d_fid,
                                qram_traj_stats *d_st, void *stream) {
  if (!d_fid) return fail(c, QRAM_E_INVAL, "d_fid is required");
  return run_mode(c, 0, seed, traj0, ntraj, d_fid, d_st, nullptr, nullptr, (hipStream_t)stream, false);
}

qram_status qram_run_pruned_async(qram_ctx *c, uint64_t seed, uint64_t traj0,
                                  uint32_t ntraj, double *d_fid,
                                  qram_traj_stats *d_st, void *stream) {
  if (!d_fid) return fail(c, QRAM_E_INVAL, "d_fid is required");
  return run_mode(c, 1, seed, traj0, ntraj, d_fid, d_st, nullptr, nullptr, (hipStream_t)stream, false);
}

qram_status qram_run_plain(qram_ctx *c, uint64_t seed, uint64_t traj0,
                           uint32_t ntraj, double *fid, qram_traj_stats *st) {
  if (!fid) return fail(c, QRAM_E_INVAL, "fid is required");
  return run_mode(c, QRAM_MODE_PLAIN, seed, traj0, ntraj, nullptr, nullptr, fid, st, c ? c->stream : nullptr, true);
}

qram_status qram_run_plain_async(qram_ctx *c, uint64_t seed, uint64_t traj0,
                                 uint32_t ntraj, double *d_fid,
                                 qram_traj_stats *d_st, void *stream) {
  if (!d_fid) return fail(c, QRAM_E_INVAL, "d_fid is required");
  return run_mode(c, QRAM_MODE_PLAIN, seed, traj0, ntraj, d_fid, d_st, nullptr, nullptr, (hipStream_t)stream, false);
}

qram_status qram_footprint(qram_ctx *c, qram_mode mode, uint32_t ntraj,
                           uint64_t *bytes) {
  if (!c || !bytes) return fail(c, QRAM_E_INVAL, "null argument");
  if (mode != QRAM_MODE_FULL && mode != QRAM_MODE_PRUNED && mode != QRAM_MODE_PLAIN) return fail(c, QRAM_E_INVAL, "bad mode");
  HIPCHK(c, hipSetDevice(c->device));
  const uint32_t nb = batch_size(c, std::max<uint32_t>(ntraj, 1u));
  Plan pl;
  qram_status st = make_plan(c, mode, nb, pl);
  if (st) return st;
  *bytes = (uint64_t)(table_bytes(c) + buffers_bytes(c, nb, pl));
  return QRAM_OK;
}

qram_status qram_reserve(qram_ctx *c, qram_mode mode, uint32_t ntraj) {
  if (!c) return QRAM_E_INVAL;
  if (mode != QRAM_MODE_FULL && mode != QRAM_MODE_PRUNED && mode != QRAM_MODE_PLAIN) return fail(c, QRAM_E_INVAL, "bad mode");
  HIPCHK(c, hipSetDevice(c->device));
  const uint32_t nb = batch_size(c, std::max<uint32_t>(ntraj, 1u));
  Plan pl;
  qram_status st = make_plan(c, mode, nb, pl);
  if (st) return st;
  return ensure_buffers(c, nb, &pl);
}

qram_status qram_errors(qram_ctx *c) {
  if (!c) return QRAM_E_INVAL;
  HIPCHK(c, hipSetDevice(c->device));
  if (c->scratch_used && c->scratch) {
    uint32_t e = 0;
    HIPCHK(c, hipMemcpy(&e, c->scratch + SCR_ERR, 4, hipMemcpyDeviceToHost));
    if (e) {
      const uint32_t z = 0;
      HIPCHK(c, hipMemcpy(c->scratch + SCR_ERR, &z, 4, hipMemcpyHostToDevice));
      if (e & ERR_CAND) return fail(c, QRAM_E_CAPACITY, "candidate buffer overflow");
      if (e & ERR_LIST) return fail(c, QRAM_E_CAPACITY, "explicit site list overflow");
    }
  }
  if (!c->errw) return QRAM_OK;
  return check_err(c);
}

qram_status qram_run_pruned_async_noalloc(qram_ctx *c, uint64_t seed, uint64_t traj0,
                                          uint32_t ntraj, double *d_fid,
                                          qram_traj_stats *d_st, void *stream) {
  if (!d_fid) return fail(c, QRAM_E_INVAL, "d_fid is required");
  qram_status st = check_args(c, traj0, ntraj);
  if (st) return st;
  if (!c->scratch) return fail(c, QRAM_E_DEVICE, "the scratch array has no address on this device");
  if (c->general)
    return fail(c, QRAM_E_INVAL, "the no-allocation entry serves contexts of the trajectory kernel (qram_create: damping, "
                                 "data-loading input, qubit k <= 6)");
  const hipStream_t s = (hipStream_t)stream;
  const int mode = 1;
  // per trajectory: candidates, five counters, digest, bad bitmap, explicit list
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const uint32_t ccap = cand_capacity(c);
  const size_t words64 = (size_t)(c->D + 63) / 64;
  auto traj_bytes = [&](size_t nb) {
    return al(nb * ccap * 4) + 5 * al(nb * 4) + al(nb * 8) + al(nb * words64 * 8) + al(nb * (size_t)c->D * 2);
  };
  const size_t avail = SCRATCH_BYTES - SCR_HEAD;
  // trajectories per batch: at most half of the array, the rest for the
  // per-workgroup pools
  uint32_t nb = std::max<uint32_t>(1u, std::min<uint32_t>(ntraj ? ntraj : 1u, 262144u));
  while (nb > 1 && traj_bytes(nb) > avail / 2) nb = (nb + 1) / 2;
  Plan pl;
  uint32_t grid_cap = 0;
  for (;;) {
    if ((st = make_plan(c, mode, nb, pl))) return st;
    size_t per_wg = al((size_t)pl.pool_slots * c->rec * 2) + al((size_t)pl.pool_slots * 4);
    per_wg += al((size_t)pl.ecap_max * 4);
    const size_t tb = traj_bytes(nb);
    grid_cap = tb < avail ? (uint32_t)std::min<size_t>((avail - tb) / per_wg, 1u << 20) : 0u;
    if (grid_cap >= 1 || nb == 1) break;
    nb = (nb + 1) / 2;
  }
  if (grid_cap < 1)
    return fail(c, QRAM_E_CAPACITY, "one workgroup's buffers exceed the " + std::to_string(SCRATCH_BYTES >> 20) +
                                         " MiB scratch array");
  pl.grid_max = 0;
  for (int i = 0; i < pl.nb; ++i) {
    pl.b[i].grid = std::min(pl.b[i].grid, grid_cap);
    pl.grid_max = std::max(pl.grid_max, pl.b[i].grid);
  }
  // carve the array
  unsigned char *base = c->scratch;
  size_t off = SCR_HEAD;
  auto take = [&](size_t bytes) {
    unsigned char *p = base + off;
    off += al(bytes);
    return p;
  };
  Run r{};
  r.seed = seed;
  r.mode = mode;
  r.cand_cap = ccap;
  r.tier2_slow = c->tier2_global ? 1u : 0u;
  r.cdec_all = pl.cdec_all ? 1u : 0u;
  r.nbkt = (uint32_t)pl.nb;
  for (int i = 0; i < pl.nb; ++i) r.bkt_emax[i] = pl.b[i].emax;
  r.pool_slots = pl.pool_slots;
  r.persistent = pl.persistent ? 1u : 0u;
  r.err = reinterpret_cast<uint32_t *>(base + SCR_ERR);
  r.counter = reinterpret_cast<uint32_t *>(base + SCR_COUNTER);
  r.bucket_base = reinterpret_cast<uint32_t *>(base + SCR_BBASE);
  r.cand = reinterpret_cast<uint32_t *>(take((size_t)nb * ccap * 4));
  r.ncand = reinterpret_cast<uint32_t *>(take((size_t)nb * 4));
  r.nbad = reinterpret_cast<uint32_t *>(take((size_t)nb * 4));
  r.ref = reinterpret_cast<uint32_t *>(take((size_t)nb * 4));
  r.nexpl = reinterpret_cast<uint32_t *>(take((size_t)nb * 4));
  r.order = reinterpret_cast<uint32_t *>(take((size_t)nb * 4));
  r.digest = reinterpret_cast<uint64_t *>(take((size_t)nb * 8));
  r.badbits = reinterpret_cast<uint64_t *>(take((size_t)nb * words64 * 8));
  r.xlist = reinterpret_cast<uint16_t *>(take((size_t)nb * c->D * 2));
  r.pool = reinterpret_cast<uint16_t *>(take((size_t)pl.grid_max * pl.pool_slots * c->rec * 2));
  r.devl = reinterpret_cast<uint32_t *>(take((size_t)pl.grid_max * pl.pool_slots * 4));
  r.gstate = reinterpret_cast<uint32_t *>(take((size_t)pl.grid_max * pl.ecap_max * 4));
  if (off > SCRATCH_BYTES) return fail(c, QRAM_E_CAPACITY, "scratch layout exceeds the array");
  c->scratch_used = true;
  // the error word starts each call at zero (a fill kernel, no memset node)
  HIPCHK(c, launch_fill_u32(r.err, 0u, 1u, s));
  for (uint32_t b0 = 0; b0 < ntraj; b0 += nb) {
    Run rb = r;
    rb.traj0 = (uint32_t)(traj0 + b0);
    rb.ntraj = std::min(nb, ntraj - b0);
    rb.fid = d_fid + b0;
    rb.st = d_st ? d_st + b0 : nullptr;
    if ((st = enqueue_batch(c, pl, rb, s, false, false, true))) return st;
  }
  return QRAM_OK;
}

qram_status qram_fidelity(const double *fid, uint32_t ntraj, double *mean,
                          double *sem) {
  if (!fid || !mean) return QRAM_E_INVAL;
  if (ntraj == 0) {
    *mean = 0.0;
    if (sem) *sem = 0.0;
    return QRAM_OK;
  }
  double m = 0.0;
  for (uint32_t i = 0; i < ntraj; ++i) m += fid[i];
  m /= ntraj;
  double v = 0.0;
  for (uint32_t i = 0; i < ntraj; ++i) v += (fid[i] - m) * (fid[i] - m);
  *mean = m;
  if (sem) *sem = ntraj > 1 ? std::sqrt(v / (ntraj - 1) / ntraj) : 0.0;
  return QRAM_OK;
}

qram_status qram_set_launch(qram_ctx *c, qram_mode mode, int slots_per_thread,
                            int schedule) {
  if (!c) return QRAM_E_INVAL;
  if (mode != QRAM_MODE_FULL && mode != QRAM_MODE_PRUNED && mode != QRAM_MODE_PLAIN)
    return fail(c, QRAM_E_INVAL, "bad mode");
  if (mode == QRAM_MODE_PLAIN || c->general) {  // workgroups per CU, threads per workgroup
    if (slots_per_thread < 0 || slots_per_thread > 32)
      return fail(c, QRAM_E_INVAL, "plain engine: 0..32 workgroups per compute unit");
    const int t = schedule & ~1;
    if (t != 0 && t != 64 && t != 128 && t != 256 && t != 512 && t != 1024)
      return fail(c, QRAM_E_INVAL,
                  "plain engine: 0, 64, 128, 256, 512 or 1024 threads per workgroup (+1: records in device memory)");
    c->plain_per_cu[mode] = slots_per_thread;
    c->plain_thr[mode] = t;
    c->plain_glob[mode] = (schedule & 1) != 0;
    c->plain_used_thr[mode] = 0;
    return QRAM_OK;
  }
  if (slots_per_thread != 0 && slots_per_thread != 4 && slots_per_thread != 8 && slots_per_thread != 16 &&
      slots_per_thread != 32 && slots_per_thread != 64)
    return fail(c, QRAM_E_INVAL, "slots_per_thread must be 0, 4, 8, 16, 32 or 64");
  if (schedule < 0 || schedule > 3) return fail(c, QRAM_E_INVAL, "schedule must be 0, 1, 2 or 3");
  c->spt[mode] = slots_per_thread;
  c->schedule[mode] = schedule;
  return QRAM_OK;
}

qram_status qram_get_launch(const qram_ctx *c, qram_mode mode,
                            int *slots_per_thread, int *schedule) {
  if (!c || !slots_per_thread || !schedule) return QRAM_E_INVAL;
  if (mode != QRAM_MODE_FULL && mode != QRAM_MODE_PRUNED && mode != QRAM_MODE_PLAIN) return QRAM_E_INVAL;
  if (mode == QRAM_MODE_PLAIN || c->general) {  // the shape in use: explicit or automatic
    int threads = 0, per_cu = 0;
    bool glob = false;
    plain_shape(c, mode, threads, per_cu, glob, 0);
    if (!c->plain_thr[mode] && c->plain_used_thr[mode]) threads = c->plain_used_thr[mode];  // (the last run's)
    const int occ = plain_occupancy(c->enc, threads, plain_lds(c, threads, glob));
    *slots_per_thread = occ > 0 ? std::min(per_cu, occ) : per_cu;
    *schedule = threads + (plain_slab(c, threads, glob) ? 0 : 1);  // (+1: records in device memory)
    return QRAM_OK;
  }
  *slots_per_thread = c->spt[mode] ? c->spt[mode] : 16;
  *schedule = c->schedule[mode];
  return QRAM_OK;
}

qram_status qram_set_option(qram_ctx *c, int option, int value) {
  if (!c) return QRAM_E_INVAL;
  if (option == QRAM_OPT_TIER2_GLOBAL) {
    c->tier2_global = value != 0;
    return QRAM_OK;
  }
  if (option == QRAM_OPT_GRAPH) {
    c->use_graph = value != 0;
    return QRAM_OK;
  }
  if (option == QRAM_OPT_SUBTREE_MARKING) {
    c->mark_subtree = value != 0;
    return QRAM_OK;
  }
  return fail(c, QRAM_E_INVAL, "unknown option");
}

qram_status qram_autotune(qram_ctx *c, qram_mode mode, uint64_t seed,
                          uint64_t traj0, uint32_t ntraj, double *best_ms) {
  qram_status st = check_args(c, traj0, ntraj);
  if (st) return st;
  if (mode != QRAM_MODE_FULL && mode != QRAM_MODE_PRUNED && mode != QRAM_MODE_PLAIN)
    return fail(c, QRAM_E_INVAL, "bad mode");
  if (ntraj == 0) return fail(c, QRAM_E_INVAL, "ntraj must be positive");
  const uint32_t nt = std::min(ntraj, batch_size(c, ntraj));
  if ((st = ensure_out(c, nt))) return st;
  if (mode == QRAM_MODE_PLAIN || c->general) {
    // the plain engine: threads per workgroup, and workgroups per compute
    // unit up to what fits
    double best = 1e300;
    int bw = 0, bt = 0;
    bool bg = false;
    const int m = mode;
    const int keep_w = c->plain_per_cu[m], keep_t = c->plain_thr[m];
    const bool keep_g = c->plain_glob[m];
    struct Shape {
      int t, w;
      bool g;
    };
    std::vector<Shape> shapes;
    for (bool g : {false, true}) {
      if (g && c->tier2_global) continue;  // (every shape keeps its records in device memory already)
      for (int t : {64, 128, 256, 512, 1024}) {
        if (t > 256 && !(c->dsplit && mode == QRAM_MODE_PRUNED)) continue;  // (large workgroups: split runs only)
        if (!g && !plain_slab(c, t, false)) continue;  // (no slab fits: the same as in device memory)
        const int occ = plain_occupancy(c->enc, t, plain_lds(c, t, g));
        if (occ < 1) continue;
        for (int w : {occ, (occ + 1) / 2, (occ + 3) / 4})
          if (shapes.empty() || shapes.back().t != t || shapes.back().w != w || shapes.back().g != g)
            shapes.push_back({t, w, g});
      }
    }
    const uint32_t ntp = std::min<uint32_t>(nt, 16384u);  // (18 shapes, 24 for a split run; two runs each)
    for (const auto &sh : shapes) {
      c->plain_thr[m] = sh.t;
      c->plain_per_cu[m] = sh.w;
      c->plain_glob[m] = sh.g;
      Plan pl;
      if (make_plan(c, mode, ntp, pl) != QRAM_OK) continue;
      if ((st = ensure_buffers(c, ntp, &pl))) return st;
      Run r = base_run(c, mode, seed, &pl);
      r.traj0 = (uint32_t)traj0;
      r.ntraj = ntp;
      r.fid = c->fid_tmp;
      r.st = nullptr;
      HIPCHK(c, launch_sample(c->dtab, r, ntp, sample_grid(c, ntp), c->stream));
      if (r.dep) HIPCHK(c, launch_sample_depol(c->dtab, r, sample_grid(c, ntp), c->stream));
      HIPCHK(c, launch_classify(c->dtab, r, ntp, sample_grid(c, ntp), c->D, c->mark_subtree, c->stream));
      double ms = 1e300;
      for (int rep = 0; rep < 2; ++rep) {  // best of two
        HIPCHK(c, hipEventRecord(c->ev[0], c->stream));
        if (pl.split) {  // a split run: its whole evolution (the plain share alone is too short to time)
          HIPCHK(c, launch_order(c->dtab, r, c->stream));
          if ((st = launch_buckets(c, pl, r, c->stream))) return st;
        }
        HIPCHK(c, launch_plain(c->dtab, r, c->enc, pl.pvar, pl.pb.grid, pl.pb.threads, pl.plds, c->stream));
        HIPCHK(c, hipEventRecord(c->ev[1], c->stream));
        HIPCHK(c, hipEventSynchronize(c->ev[1]));
        float t;
        HIPCHK(c, hipEventElapsedTime(&t, c->ev[0], c->ev[1]));
        ms = std::min(ms, (double)t);
      }
      if (ms < best) {
        best = ms;
        bw = sh.w;
        bt = sh.t;
        bg = sh.g;
      }
    }
    c->plain_per_cu[m] = bw ? bw : keep_w;
    c->plain_thr[m] = bt ? bt : keep_t;
    c->plain_glob[m] = bw ? bg : keep_g;
    if (best_ms) *best_ms = best;
    return check_err(c);
  }
  const int cands[5] = {4, 8, 16, 32, 64};
  double best = 1e300;
  int bs = 16, bsched = 1;
  bool sampled = false;
  for (int sched = 0; sched < 4; ++sched) {
    for (int ci = 0; ci < 5; ++ci) {
      c->spt[mode] = cands[ci];
      c->schedule[mode] = sched;
      Plan pl;
      if (make_plan(c, mode, nt, pl) != QRAM_OK) continue;
      if ((st = ensure_buffers(c, nt, &pl))) return st;
      Run r = base_run(c, mode, seed, &pl);
      r.traj0 = (uint32_t)traj0;
      r.ntraj = nt;
      r.fid = c->fid_tmp;
      r.st = nullptr;
      if (!sampled) {
        HIPCHK(c, launch_sample(c->dtab, r, nt, sample_grid(c, nt), c->stream));
        sampled = true;
      }
      double t_best = 1e300;
      for (int rep = 0; rep < 2; ++rep) {
        HIPCHK(c, launch_classify(c->dtab, r, nt, sample_grid(c, nt), c->D, c->mark_subtree, c->stream));
        HIPCHK(c, launch_order(c->dtab, r, c->stream));
        HIPCHK(c, hipEventRecord(c->ev[0], c->stream));
        if ((st = launch_buckets(c, pl, r, c->stream))) return st;
        HIPCHK(c, hipEventRecord(c->ev[1], c->stream));
        HIPCHK(c, hipEventSynchronize(c->ev[1]));
        float ms;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev[0], c->ev[1]));
        t_best = std::min(t_best, (double)ms);
      }
      // state words in device memory must beat shared memory by 3% to be
      // chosen: within that they only add HBM traffic (other work on the
      // device pays for it)
      const double score = (sched & 2) ? t_best * 1.03 : t_best;
      if (score < best) {
        best = score;
        bs = cands[ci];
        bsched = sched;
      }
    }
  }
  c->spt[mode] = bs;
  c->schedule[mode] = bsched;
  if (best_ms) *best_ms = (bsched & 2) ? best / 1.03 : best;
  return check_err(c);
}

qram_status qram_last_kernel_ms(const qram_ctx *c, double *times) {
  if (!c || !times) return QRAM_E_INVAL;
  for (int i = 0; i < 3; ++i) times[i] = c->last_ms[i];
  return QRAM_OK;
}

qram_status qram_set_timing(qram_ctx *c, int on) {
  if (!c) return QRAM_E_INVAL;
  c->timing = on != 0;
  c->tev_used = 0;
  c->tev_launches = 0;
  c->tev_nb.clear();
  return QRAM_OK;
}

qram_status qram_stage_buckets(qram_ctx *c, double *ms, uint32_t *launches, uint32_t *ntraj_last,
                               uint32_t *emax, int *nbuckets) {
  if (!c || !ms || !launches || !ntraj_last || !emax || !nbuckets) return QRAM_E_INVAL;
  HIPCHK(c, hipSetDevice(c->device));
  for (int i = 0; i < MAXB; ++i) {
    ms[i] = 0.0;
    launches[i] = ntraj_last[i] = emax[i] = 0;
  }
  const size_t nb = c->tev_used / EVB;
  int nbk = 0;
  for (size_t b = 0; b < nb; ++b) {
    const int k = c->tev_nb[b];
    nbk = std::max(nbk, k);
    for (int i = 0; i < k; ++i) {
      HIPCHK(c, hipEventSynchronize(c->tev[EVB * b + 5 + 2 * i]));
      float t;
      HIPCHK(c, hipEventElapsedTime(&t, c->tev[EVB * b + 4 + 2 * i], c->tev[EVB * b + 5 + 2 * i]));
      ms[i] += t;
      launches[i] += 1;
    }
  }
  if (nb && c->bucket_base && nbk > 0) {  // trajectories per bucket in the last timed batch
    uint32_t bb[MAXB + 1];
    HIPCHK(c, hipMemcpy(bb, c->bucket_base, sizeof(bb), hipMemcpyDeviceToHost));
    for (int i = 0; i < nbk; ++i) ntraj_last[i] = bb[i + 1] - bb[i];
  }
  for (int i = 0; i < MAXB; ++i) emax[i] = c->tev_emax[i];
  *nbuckets = nbk;
  return QRAM_OK;
}

qram_status qram_stage_launches(const qram_ctx *c, uint32_t *evolve_launches) {
  if (!c || !evolve_launches) return QRAM_E_INVAL;
  *evolve_launches = c->tev_launches;
  return QRAM_OK;
}

qram_status qram_stage_times(qram_ctx *c, double *ms, uint32_t *nbatches) {
  if (!c || !ms) return QRAM_E_INVAL;
  HIPCHK(c, hipSetDevice(c->device));
  ms[0] = ms[1] = ms[2] = 0.0;
  const size_t nb = c->tev_used / EVB;
  for (size_t b = 0; b < nb; ++b) {
    HIPCHK(c, hipEventSynchronize(c->tev[EVB * b + 3]));
    for (int i = 0; i < 3; ++i) {
      float t;
      HIPCHK(c, hipEventElapsedTime(&t, c->tev[EVB * b + i], c->tev[EVB * b + i + 1]));
      ms[i] += t;
    }
  }
  if (nbatches) *nbatches = (uint32_t)nb;
  c->tev_used = 0;
  c->tev_launches = 0;
  c->tev_nb.clear();
  return QRAM_OK;
}

// One trajectory, sampled from (seed, traj) or under a forced history,
// optionally exporting its final components and its jump log.
static qram_status run_single(qram_ctx *c, int mode, uint64_t seed, uint32_t traj, bool forced,
                              const uint32_t *cand_L, uint32_t ncand, const double *u_aux, double u_fin,
                              uint32_t *h_exp, uint32_t exp_cap, double *h_amp, uint32_t *h_jlog, uint32_t jcap,
                              uint32_t *h_njl, double *fid, qram_traj_stats *stt) {
  qram_status st = check_args(c, traj, 1);
  if (st) return st;
  if (mode != QRAM_MODE_FULL && mode != QRAM_MODE_PRUNED && mode != QRAM_MODE_PLAIN) return fail(c, QRAM_E_INVAL, "bad mode");
  if (!fid) return fail(c, QRAM_E_INVAL, "null argument");
  if (forced) {
    if (!u_aux || (ncand && !cand_L)) return fail(c, QRAM_E_INVAL, "null argument");
    const uint64_t S = (uint64_t)(c->T - 1) * c->M;
    for (uint32_t j = 0; j < ncand; ++j) {
      if (cand_L[j] >= S) return fail(c, QRAM_E_INVAL, "candidate index out of range");
      if (j && cand_L[j] <= cand_L[j - 1]) return fail(c, QRAM_E_INVAL, "candidates must be strictly ascending");
    }
  }
  const size_t rec_words = 3 + (size_t)c->lmax;
  const size_t ncomp = (size_t)c->D * c->K2;
  if (h_exp && exp_cap < ncomp) return fail(c, QRAM_E_CAPACITY, "the export needs one record per component (2^n * 2^k or 2^n)");
  Plan pl;
  if ((st = make_plan(c, mode, 1, pl, false))) return st;
  if ((st = ensure_buffers(c, 1, &pl))) return st;
  if (forced && ncand > c->cand_cap) {
    if ((st = dev_alloc(c, &c->cand, ncand))) return st;
    c->cand_cap = ncand;
    c->batch_cap = 1;
  }
  if ((st = ensure_out(c, 1))) return st;
  Run r = base_run(c, mode, seed, &pl);
  r.traj0 = traj;
  r.ntraj = 1;
  if (forced) {
    if (!c->uaux)
      if ((st = dev_alloc(c, &c->uaux, MAXT))) return st;
    std::vector<double> ua(MAXT, 0.0);
    for (int s = 0; s < c->T; ++s) ua[s] = u_aux[s];
    HIPCHK(c, hipMemcpy(c->uaux, ua.data(), MAXT * 8, hipMemcpyHostToDevice));
    if (ncand) HIPCHK(c, hipMemcpy(c->cand, cand_L, ncand * 4, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->ncand, &ncand, 4, hipMemcpyHostToDevice));
    r.forced = 1;  // (depolarizing faults are still drawn for (seed, traj))
    r.uaux = c->uaux;
    r.ufin = u_fin;
  }
  if (h_exp) {
    if ((st = grow(c, &c->dexp, &c->dexp_cap, ncomp * rec_words))) return st;
    HIPCHK(c, hipMemsetAsync(c->dexp, 0, ncomp * rec_words * 4, c->stream));
    r.exp = c->dexp;
    if (pl.plain) {
      if ((st = grow(c, &c->dexpamp, &c->dexpamp_cap, ncomp * 2))) return st;
      HIPCHK(c, hipMemsetAsync(c->dexpamp, 0, ncomp * 16, c->stream));
      r.expamp = c->dexpamp;
    }
  }
  if (h_njl) {
    if ((st = grow(c, &c->djlog, &c->djlog_cap, std::max<size_t>(jcap, 1)))) return st;
    if ((st = grow(c, &c->djn, &c->djn_cap, 1))) return st;
    r.jlog = c->djlog;
    r.jn = c->djn;
    r.jcap = jcap;
  }
  r.fid = c->fid_tmp;
  r.st = c->st_tmp;
  if ((st = enqueue_batch(c, pl, r, c->stream, false, forced))) return st;
  HIPCHK(c, hipMemcpyAsync(fid, c->fid_tmp, 8, hipMemcpyDeviceToHost, c->stream));
  if (stt) HIPCHK(c, hipMemcpyAsync(stt, c->st_tmp, sizeof(qram_traj_stats), hipMemcpyDeviceToHost, c->stream));
  if (h_exp)
    HIPCHK(c, hipMemcpyAsync(h_exp, c->dexp, ncomp * rec_words * 4, hipMemcpyDeviceToHost, c->stream));
  if (h_exp && h_amp && pl.plain)
    HIPCHK(c, hipMemcpyAsync(h_amp, c->dexpamp, ncomp * 16, hipMemcpyDeviceToHost, c->stream));
  if (h_njl) {
    HIPCHK(c, hipMemcpyAsync(h_njl, c->djn, 4, hipMemcpyDeviceToHost, c->stream));
    if (jcap && h_jlog) HIPCHK(c, hipMemcpyAsync(h_jlog, c->djlog, (size_t)jcap * 4, hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return check_err(c);
}

qram_status qram_run_forced(qram_ctx *c, qram_mode mode, const uint32_t *cand_L,
                            uint32_t ncand, const double *u_aux, double u_fin,
                            double *fid, qram_traj_stats *stt) {
  return run_single(c, mode, 0, 0, true, cand_L, ncand, u_aux, u_fin, nullptr, 0, nullptr, nullptr, 0, nullptr, fid,
                    stt);
}

qram_status qram_export_state(qram_ctx *c, qram_mode mode, uint64_t seed, uint32_t traj,
                              const uint32_t *cand_L, uint32_t ncand, const double *u_aux,
                              double u_fin, uint32_t *comp, uint32_t comp_cap, double *amp,
                              uint32_t *jlog, uint32_t jcap, uint32_t *njl, double *fid,
                              qram_traj_stats *stt) {
  if (!comp || !njl) return fail(c, QRAM_E_INVAL, "comp and njl are required");
  if (c && (mode == QRAM_MODE_PLAIN || c->general) && !amp)
    return fail(c, QRAM_E_INVAL, "the plain engine exports amplitudes: amp is required");
  return run_single(c, mode, seed, traj, u_aux != nullptr, cand_L, ncand, u_aux, u_fin, comp, comp_cap, amp, jlog,
                    jcap, njl, fid, stt);
}

qram_status qram_run_jumplog(qram_ctx *c, qram_mode mode, uint64_t seed, uint64_t traj0,
                             uint32_t ntraj, double *fid, qram_traj_stats *stt, uint32_t *jlog,
                             uint32_t jcap, uint32_t *njl) {
  if (!c) return fail(nullptr, QRAM_E_INVAL, "null context");
  if (mode != QRAM_MODE_FULL && mode != QRAM_MODE_PRUNED && mode != QRAM_MODE_PLAIN) return fail(c, QRAM_E_INVAL, "bad mode");
  if (!fid || !njl || (jcap && !jlog)) return fail(c, QRAM_E_INVAL, "null argument");
  return run_mode(c, (int)mode, seed, traj0, ntraj, nullptr, nullptr, fid, stt, c->stream, true, jlog, jcap, njl);
}

qram_status qram_dense_dim(const qram_ctx *c, uint64_t *N) {
  if (!c || !N) return QRAM_E_INVAL;
  *N = dense_dim(c->n, c->k, c->enc);
  return QRAM_OK;
}

static DenseJob dense_job(const qram_ctx *c, double dephase, double heat) {
  DenseJob j;
  j.n = c->n;
  j.k = c->k;
  j.enc = c->enc;
  j.gamma = c->gamma;
  j.eps = c->eps;
  j.dephase = dephase;
  j.heat = heat;
  j.mem = c->mem;
  j.in_idx = c->in_idx;
  j.in_amp = c->in_amp;
  return j;
}

qram_status qram_dense_density(qram_ctx *c, double dephase, double heat, double *F_rho, double *trace) {
  if (!c || !F_rho || !trace) return fail(c, QRAM_E_INVAL, "null argument");
  if (!(dephase >= 0.0 && dephase <= 1.0) || !(heat >= 0.0 && heat <= 1.0))
    return fail(c, QRAM_E_INVAL, "dephase and heat must lie in [0, 1]");
  if (dense_dim(c->n, c->k, c->enc) > 4096) return fail(c, QRAM_E_RANGE, "density matrix: at most 4096 basis states (n <= 2)");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, dense_density(c->dtab, dense_job(c, dephase, heat), c->stream, F_rho, trace));
  return QRAM_OK;
}

qram_status qram_dense_forced(qram_ctx *c, const uint32_t *jumps, uint32_t njumps, const uint32_t *faults,
                              uint32_t nfaults, double *psi, uint64_t cap) {
  if (!c || !psi || (njumps && !jumps) || (nfaults && !faults)) return fail(c, QRAM_E_INVAL, "null argument");
  const uint64_t N = dense_dim(c->n, c->k, c->enc);
  if (c->n > 3 || N > (1ull << 25)) return fail(c, QRAM_E_RANGE, "dense state: n <= 3 and at most 2^25 basis states");
  if (cap < N) return fail(c, QRAM_E_CAPACITY, "psi needs 2 * N doubles (qram_dense_dim)");
  uint32_t prev = 0;
  for (uint32_t t = 0; t < njumps; ++t) {
    const uint32_t s = jumps[t] >> 24, q = jumps[t] & 0xFFFFu, lev = (jumps[t] >> 16) & 0xFFu;
    const uint32_t levmax = (c->enc == QUTRIT && (q & 1u) == 0) ? 2u : 1u;
    if (s < 1 || s >= (uint32_t)c->T || s < prev || q >= (uint32_t)c->M || lev < 1 || lev > levmax)
      return fail(c, QRAM_E_INVAL, "jumps: site | level << 16 | slice << 24, slices ascending in 1..T-1");
    prev = s;
  }
  prev = 0;
  for (uint32_t t = 0; t < nfaults; ++t) {
    const uint32_t s = (faults[t] >> 16) & 0xFFu, q = faults[t] & 0xFFFFu, ty = faults[t] >> 24;
    const uint32_t d = (c->enc == QUTRIT && (q & 1u) == 0) ? 3u : 2u;
    if (s < 1 || s >= (uint32_t)c->T || s < prev || q >= (uint32_t)c->M || (ty & 3u) >= d || (ty >> 2) >= d)
      return fail(c, QRAM_E_INVAL, "faults: site | slice << 16 | type << 24, slices ascending in 1..T-1");
    prev = s;
  }
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, dense_forced(c->dtab, dense_job(c, 0.0, 0.0), jumps, njumps, faults, nfaults, c->stream, psi));
  return QRAM_OK;
}

}  // extern "C"
