// Internal declarations shared by the host code and the kernels of the HIP
// library.  Nothing here is visible through the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/qram.h"

namespace qr {

constexpr int MAXN = 15;
constexpr int MAXK = 8;
constexpr int MAXT = 6 * MAXN + 2 * MAXK + 1;  // slices 0..T
constexpr uint8_t NONE = 0xFF;
constexpr int NCS = 16;    // a slice with at most NCS candidates is scanned as a list
constexpr int JMAX = 64;   // joint outcome capacity (|J| <= excitations of one component)
constexpr int MAXB = 6;    // work buckets of the evolution launches
constexpr int MAXSPT = 64; // component slots per thread (one bit each in a mask)
constexpr int QUTRIT = 0;
constexpr int QUBIT = 1;

// State word of an explicit component.  Its slot fixes its initial label
// (address, bus word).  Tier 1 (no jump has touched its routing):
//   bits  0..7  exposure carried by data tokens it lost
//   bits  8..15 live data tokens (qubit: bus bits still carried; qutrit:
//               data bits not yet lost)
// Tier 2 (explicit site list in the pool):
//   bits  0..15 exposure through the previous slice
//   bits 16..23 excited sites now (the record's count); after the last
//               slice, with bit 27 set, the bus word of a ground list
//   bit  27     ground after the last slice, bits 16..23 hold the bus word
//   bit  28     a candidate of this slice sits on one of its sites
//   bit  29     qubit: the address's components keep one list each (else
//               the address's bus words share one list)
// Both: bit 24 sign, bit 25 alive, bit 26 tier 2.
constexpr uint32_t W_EK = 0xFFu;
constexpr int W_LIVE_SH = 8;
constexpr uint32_t W_E = 0xFFFFu;
constexpr int W_CNT_SH = 16;
constexpr uint32_t W_CNT = 0xFFu << W_CNT_SH;
constexpr uint32_t W_SIGN = 1u << 24;
constexpr uint32_t W_ALIVE = 1u << 25;
constexpr uint32_t W_DEV = 1u << 26;
constexpr uint32_t W_FBUS = 1u << 27;
constexpr uint32_t W_HIT = 1u << 28;
constexpr uint32_t W_SPLIT = 1u << 29;  // qubit tier 2: the address keeps one list per component

// Tier-2 record in the pool (uint16 words): [0] count, [1] bus word,
// [2..] excited sites.  Qutrit router sites carry their level in bit 15
// (set: R, clear: L).
constexpr uint16_t LV_R_BIT = 0x8000u;
// Largest evolution workgroup of each encoding.
constexpr int EVOLVE_MAX_THREADS[2] = {512, 1024};

struct Tables {
  int n, k, enc, T, M, D, K2, lmax, emax, rec;  // rec = pool record length (even)
  uint64_t G[64];                 // geometric-walk thresholds
  const uint32_t *mem;            // [D] memory words
  const double *wpow;             // [emax + max(emax, prec) + 1] (1-gamma)^(m - emax)
  const double *apow;             // [emax + max(emax, prec) + 1] a^(m - emax)
  const double *ftab_w;           // [(T + 1) * nfs] per-slice factor tables, (1-gamma)^e
  const double *ftab_a;           // the same with a^e
  int nfs;                        // entries per slice: 96 address-chunk, 2^k data, 1 router
  const double *ctot;             // [T] total no-jump weight of all addresses through slice s
  double ov_nojump, w_nojump;     // final overlap and weight when no jump occurred
  uint32_t amask[MAXT];  // address tokens excitable after the gates of s (bit n-1-t)
  uint32_t dmask[MAXT];  // data tokens excitable after the gates of s (bit b)
  uint32_t cswap[MAXT];  // layers whose controlled swap fires at s
  uint8_t nrouter[MAXT]; // qutrit: stored routers at s (always excited)
  int8_t copy_t[MAXT], store_l[MAXT], bus_b[MAXT], fetch_b[MAXT];
  uint8_t tok[MAXT][MAXN][2];      // token at (layer, slot) of the path at s
  uint8_t pos[MAXT][MAXN + MAXK];  // layer << 1 | slot of each token at s
  uint16_t cntA[MAXT][MAXN];       // exposure of address token t through s
  uint16_t cntD[MAXT][MAXK];       // exposure of data token b through s
  uint16_t cntR[MAXT];             // qutrit: router exposure through s
  double sg;                       // sqrt(gamma), the amplitude of a jump
  // depolarizing faults (eps > 0): active positions of slice s are the sites
  // 0 .. dep_off[s+1]-dep_off[s]-1; geometric-walk thresholds for eps
  int depol;                       // 1 if eps > 0
  uint64_t Gp[64];
  uint32_t dep_off[MAXT + 1];      // linear index of slice s's first active position
  // general input (null: uniform amplitudes, bus word 0)
  const double *cin;               // [2 D] normalised amplitude (re, im) of each address
  const uint32_t *jin;             // [D] bus word of each address
  // input with amplitudes on (address, bus word) pairs: cin/jin then hold
  // the amplitude and bus word of each address holding one bus word (0
  // for the others)
  const double *cab;               // [2 D 2^k] normalised c_ij, address-major
  const double *camp;              // [2 D K2] amplitude of each component after the first wall
  const uint8_t *aflag;            // [D] bit 0: the input holds the address; bit 1: with one bus word
  int trunc_w;                     // Hamming truncation of the predicted good branches (-1: none)
};

struct Run {
  uint64_t seed;
  uint32_t traj0, ntraj;
  int mode;              // 0 full, 1 pruned
  uint32_t cand_cap;     // candidate slots per trajectory
  uint32_t forced;       // 1: forced history (single trajectory)
  uint32_t tier2_slow;   // 1: every tier-2 list takes the global-memory path
  uint32_t cdec_all;     // 1: all candidates of a trajectory fit shared memory
  // bucket of this evolution launch
  uint32_t bucket;       // index of the bucket this launch serves
  uint32_t apt;          // explicit addresses per thread
  uint32_t e_cap;        // tier-1 words per workgroup (spt * threads)
  uint32_t pool_slots;   // tier-2 records per workgroup
  uint32_t persistent;   // 1: dynamic queue, 0: static round robin
  uint32_t nbkt;         // buckets in use
  uint32_t bkt_emax[MAXB];  // explicit components admitted by each bucket
  uint32_t *cand;        // [ntraj * cand_cap] ascending L
  uint32_t *ncand;       // [ntraj]
  uint64_t *digest;      // [ntraj]
  uint64_t *badbits;     // [ntraj * words64]
  uint32_t *nbad;        // [ntraj]
  uint32_t *ref;         // [ntraj]
  uint16_t *xlist;       // [ntraj * D] explicit addresses (pruned)
  uint32_t *nexpl;       // [ntraj] explicit components
  uint32_t *order;       // [ntraj] trajectories grouped by bucket
  uint32_t *bucket_base; // [MAXB + 2] (the last: end of a split run's plain-engine segment)
  uint32_t *counter;     // [MAXB] queue heads
  uint32_t *gstate;      // [grid * e_cap] tier-1 words when not in LDS
  uint16_t *pool;        // [grid * pool_slots * rec] tier-2 records
  uint32_t *devl;        // [grid * pool_slots] tier-2 work list: component | address << 16
  double *fid;           // [ntraj]
  qram_traj_stats *st;   // [ntraj] or null
  uint32_t *err;         // [1] error bits
  const double *uaux;    // forced auxiliary uniforms [T]
  double ufin;           // forced final uniform
  // test entries (null otherwise)
  uint32_t *exp;         // [D * K2 * (3 + lmax)] component records of trajectory 0
  uint32_t *jlog;        // [ntraj * jcap] jump log: site | level << 16 | slice << 24
  uint32_t *jn;          // [ntraj] jump-log entries of each trajectory (may exceed jcap)
  uint32_t jcap;         // jump-log entries kept per trajectory
  double *expamp;        // [D * K2 * 2] plain mode: amplitude of each exported record
  // depolarizing faults of each trajectory: site | slice << 16 | type << 24
  // (type a | b << 2, the operator Z^b X^a), ascending slice and site
  uint32_t *dep;         // [ntraj * dep_cap]
  uint32_t *ndep;        // [ntraj]
  uint32_t dep_cap;
  // plain full evolution: per-workgroup component lists (pool, prec uint16
  // words each), amplitudes, hit flags and finalize scratch
  uint32_t prec;
  uint32_t pslab;        // words of each thread's record slab in shared memory (0: none)
  // 1 (pruned runs with depolarizing noise): the trajectory kernel takes the
  // trajectories that drew no depolarizing fault (ndep 0), the plain engine
  // the others, which k_order lists after every bucket
  uint32_t dsplit;
  double *pamp;          // [grid * E * 2]
  uint8_t *phit;         // [grid * E]
  double *pgrp;          // [grid * threads * K2 * 2]
};

// Export record of one component (test entry), (3 + lmax) words:
// [0] address | bus word << 16 | sign << 24 | 1 << 25, [1] exposure e (the
// amplitude is c_i * K2^(-1/2) * (-1)^sign * gamma^(|J_all|/2) * a^e, with
// |J_all| the trajectory's jump-log length), [2] excited sites,
// [3 + j] site | level << 16 (level 1: excited qubit, qutrit L or data
// qubit; 2: qutrit R).
constexpr uint32_t EXP_PRESENT = 1u << 25;

constexpr uint32_t ERR_CAND = 1u;
constexpr uint32_t ERR_LIST = 2u;

// Kernel launchers.
hipError_t launch_sample(const Tables *tb, const Run &rp, uint32_t ntraj,
                         uint32_t grid, hipStream_t s);
hipError_t launch_classify(const Tables *tb, const Run &rp, uint32_t ntraj,
                           uint32_t grid, int D, bool subtree, hipStream_t s);
hipError_t launch_order(const Tables *tb, const Run &rp, hipStream_t s);
hipError_t launch_evolve(const Tables *tb, const Run &rp, int enc,
                         uint32_t grid, int threads, uint32_t lds_bytes,
                         bool state_lds, hipStream_t s);
hipError_t launch_digest(const Run &rp, uint32_t ntraj, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, uint32_t n, hipStream_t s);
hipError_t launch_sample_depol(const Tables *tb, const Run &rp, uint32_t grid, hipStream_t s);
constexpr uint32_t ERR_DEP = 4u;  // depolarizing fault buffer overflow

uint32_t evolve_lds_bytes(int M, int D, int threads, uint32_t cdec_cap,
                          uint32_t e_cap, bool state_lds, uint32_t walk_bytes);
// Shared memory of the no-jump walk's exposure-count table: one byte per
// slice and token.
__host__ __device__ inline uint32_t walk_table_bytes(int T, int n, int k) {
  return (uint32_t)(T * (n + k));
}
int evolve_occupancy(int enc, bool state_lds, int threads, uint32_t lds_bytes);
// plain full evolution (every component explicit, slice by slice)
constexpr int PLAIN_THREADS = 256;  // (largest plain-engine workgroup)
constexpr double PLAIN_POOL_BYTES = 16.0 * 1024 * 1024 * 1024;  // plain-engine state of one launch
constexpr uint32_t PLAIN_SLAB_BYTES = 40 * 1024;  // per-workgroup record slabs in shared memory, at most
constexpr int PLAIN_EXTRA = 8;  // list entries beyond the excitation bound
uint32_t plain_lds_bytes(int M, uint32_t slab_words);
// the most plain-engine workgroups of `threads` a compute unit holds, over
// the kernel's register budgets
int plain_occupancy(int enc, int threads, uint32_t lds_bytes);
// the register budget for a launch asking for per_cu workgroups per compute
// unit (occ: how many it holds)
int plain_variant(int enc, int threads, uint32_t lds_bytes, int per_cu, int &occ);
// lets the plain kernel's large workgroups take up to lds_max bytes of
// shared memory
hipError_t plain_prepare(int lds_max);
hipError_t launch_plain(const Tables *tb, const Run &rp, int enc, int variant, uint32_t grid, int threads,
                        uint32_t lds_bytes,
                        hipStream_t s);
hipError_t evolve_prepare(int lds_max, int *dyn_max);

// dense whole-register cross-check (tiny trees)
constexpr int DENSE_MAXD = 24;  // digits: n + k + 2 (2^n - 1)
struct DenseJob {
  int n, k, enc;
  double gamma, eps, dephase, heat;
  std::vector<uint32_t> mem;     // [2^n] memory words
  std::vector<uint32_t> in_idx;  // address << 8 | bus word of each input pair
  std::vector<double> in_amp;    // its normalised amplitude (re, im)
};
uint64_t dense_dim(int n, int k, int enc);
hipError_t dense_density(const Tables *dtab, const DenseJob &job, hipStream_t st, double *F, double *tr);
hipError_t dense_forced(const Tables *dtab, const DenseJob &job, const uint32_t *jumps, uint32_t njumps,
                        const uint32_t *faults, uint32_t nfaults, hipStream_t st, double *psi_host);

}  // namespace qr
