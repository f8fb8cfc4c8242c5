// HIP kernels (gfx950) of the damped bucket-brigade QRAM trajectory simulator.
//
//   k_sample    candidate history of each trajectory (Sec. IV D, first step of
//               the joint sampler): i.i.d. Bernoulli(gamma) site-slices drawn by
//               a geometric walk over 64-site blocks, Philox4x32-10 counters.
//   k_classify  bad-address set of the marking rule (Eq. subtree / Eq.
//               badrange), reference = smallest good address, and the ascending
//               list of explicitly evolved addresses (Alg. 1 steps 1-2).
//   k_order     longest-first processing order by explicit work.
//   k_evolve    one workgroup per trajectory: every explicit component is
//               carried slice by slice through the schedule's gates and one
//               joint damping layer per slice (Eq. layerkraus, Theorem 4 with
//               the mask weights of Eq. maskweight, good-branch weights
//               included in pruned mode), then the second wall, the tree
//               measurement and the fidelity (Alg. 1 steps 3-6).
//
// Component representation in k_evolve.  A component never splits between
// the walls (every gate permutes basis labels and K_J maps survivors one to
// one), so it keeps its slot, which encodes its initial label (address, bus
// word).  While no jump has touched its routing ("tier 1") its excited sites
// are the schedule positions of its live tokens on its own path, so its state
// is one 32-bit word: exposure count, live data tokens, sign, flags.  A jump
// that removes an address token or a router changes later routing; the
// component then moves to an explicit site list ("tier 2") in a per-workgroup
// pool and follows the gates literally.  Amplitudes are c_i * sign *
// gamma^{|J|/2} * a^e; gamma^{|J|/2} is common to all survivors and cancels in
// every ratio, so each draw uses the weights (1-gamma)^e from a table.
#include "qram_internal.h"

namespace qr {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

__device__ __forceinline__ double uniform53(uint64_t seed, uint32_t c0,
                                            uint32_t c1, uint32_t traj,
                                            uint32_t tag) {
  const uint4 w = philox10(make_uint4(c0, c1, traj, tag), (uint32_t)seed,
                           (uint32_t)(seed >> 32));
  const uint64_t u = (uint64_t)w.x | ((uint64_t)w.y << 32);
  return (double)(u >> 11) * 0x1.0p-53;
}

__device__ __forceinline__ int layer_of(uint32_t v) { return 31 - __clz(v + 1); }

// ---------------------------------------------------------------------------
// Deterministic block reductions: xor butterfly inside a wave, then the wave
// partials summed in wave order by every thread.
// ---------------------------------------------------------------------------
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double *buf) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double x = v[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    v[i] = x;
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) buf[wave * N + i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += buf[w * N + i];
    v[i] = t;
  }
}

// Exclusive prefix sum of one double over the block, in thread order.
__device__ __forceinline__ double block_excl_scan(double x, double *buf) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  double incl = x;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 63) buf[wave] = incl;
  __syncthreads();
  double base = 0.0;
  for (int w = 0; w < wave; ++w) base += buf[w];
  return base + incl - x;
}

__device__ __forceinline__ uint32_t block_excl_scan_u32(uint32_t x,
                                                        uint32_t *buf,
                                                        uint32_t *total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  uint32_t incl = x;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 63) buf[wave] = incl;
  __syncthreads();
  uint32_t base = 0, tot = 0;
  for (int w = 0; w < nw; ++w) {
    if (w < wave) base += buf[w];
    tot += buf[w];
  }
  *total = tot;
  return base + incl - x;
}

// ---------------------------------------------------------------------------
// k_sample
// ---------------------------------------------------------------------------
template <bool WRITE>
__device__ __forceinline__ uint32_t walk_block(uint32_t b, uint32_t len,
                                               uint32_t traj, uint32_t k0,
                                               uint32_t k1, const uint64_t *G,
                                               uint32_t *out, uint32_t base,
                                               uint32_t cap) {
  uint32_t pos = 0, cnt = 0;
  for (uint32_t j = 0;; ++j) {
    const uint4 w = philox10(make_uint4(b, j, traj, 1u), k0, k1);
    const uint64_t u = (uint64_t)w.x | ((uint64_t)w.y << 32);
    const uint32_t rem = len - pos;  // >= 1
    // smallest gap o with u < G[o]; the walk ends when o >= rem (or none)
    if (!(u < G[rem - 1])) break;
    uint32_t lo = 0, hi = rem - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (u < G[mid])
        hi = mid;
      else
        lo = mid + 1;
    }
    if (WRITE && base + cnt < cap) out[base + cnt] = 64u * b + pos + lo;
    ++cnt;
    pos += lo + 1;
    if (pos >= len) break;
  }
  return cnt;
}

__global__ void __launch_bounds__(256) k_sample(const Tables *__restrict__ tb,
                                                const Run R_) {
  const Run *rp = &R_;
  __shared__ uint64_t G[64];
  __shared__ uint32_t sbuf[4];
  const int tid = threadIdx.x, nthr = blockDim.x;
  if (tid < 64) G[tid] = tb->G[tid];
  __syncthreads();
  const uint32_t M = tb->M, T = tb->T;
  const uint64_t S = (uint64_t)(T - 1) * M;
  const uint32_t nb = (uint32_t)((S + 63) / 64);
  const uint32_t per = (nb + nthr - 1) / nthr;
  const uint32_t b0 = min(nb, tid * per), b1 = min(nb, b0 + per);
  const uint32_t k0 = (uint32_t)rp->seed, k1 = (uint32_t)(rp->seed >> 32);
  const uint32_t cap = rp->cand_cap;
  for (uint32_t tj = blockIdx.x; tj < rp->ntraj; tj += gridDim.x) {
    const uint32_t traj = rp->traj0 + tj;
    uint32_t cnt = 0;
    for (uint32_t b = b0; b < b1; ++b) {
      const uint32_t len = (uint32_t)min((uint64_t)64, S - 64ull * b);
      cnt += walk_block<false>(b, len, traj, k0, k1, G, nullptr, 0, 0);
    }
    uint32_t total;
    const uint32_t off = block_excl_scan_u32(cnt, sbuf, &total);
    uint32_t *out = rp->cand + (size_t)tj * cap;
    if (cnt) {
      uint32_t o = off;
      for (uint32_t b = b0; b < b1; ++b) {
        const uint32_t len = (uint32_t)min((uint64_t)64, S - 64ull * b);
        o += walk_block<true>(b, len, traj, k0, k1, G, out, o, cap);
      }
    }
    if (tid == 0) {
      rp->ncand[tj] = total;
      if (total > cap) atomicOr(rp->err, ERR_CAND);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// k_classify: marks the range node of every candidate, propagates marks down
// the tree, and derives the bad bitmap, the reference and the explicit list.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t range_node(int enc, uint32_t v) {
  if (enc == QUTRIT) return v;  // Eq. subtree
  // Eq. badrange: a left child below the root's children inherits its
  // parent's range; right children and the root's children mark their own
  // subtree; the root marks everything.
  while (v > 2 && (v & 1u)) v = (v - 1) >> 1;
  return v;
}

__global__ void __launch_bounds__(256) k_classify(const Tables *__restrict__ tb,
                                                  const Run R_) {
  const Run *rp = &R_;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int n = tb->n, D = tb->D, M = tb->M, enc = tb->enc;
  const int nw32 = (D + 31) >> 5;
  uint32_t *badw = reinterpret_cast<uint32_t *>(smem);  // [nw32]
  uint32_t *sbuf = badw + nw32;                         // [16]
  uint8_t *mark = reinterpret_cast<uint8_t *>(sbuf + 16);  // [D - 1]
  const uint32_t cap = rp->cand_cap;
  const int kb = enc == QUBIT ? tb->k : 0;
  for (uint32_t tj = blockIdx.x; tj < rp->ntraj; tj += gridDim.x) {
    for (int v = tid; v < D - 1; v += nthr) mark[v] = 0;
    if (tid == 0) sbuf[8] = 0xFFFFFFFFu;
    __syncthreads();
    const uint32_t nc = min(rp->ncand[tj], cap);
    const uint32_t *cand = rp->cand + (size_t)tj * cap;
    for (uint32_t j = tid; j < nc; j += nthr) {
      const uint32_t q = cand[j] % (uint32_t)M;
      mark[range_node(enc, q >> 1)] = 1;
    }
    __syncthreads();
    for (int l = 1; l < n; ++l) {  // a node is bad if it or an ancestor is marked
      const int v0 = (1 << l) - 1;
      for (int v = v0 + tid; v < 2 * v0 + 1; v += nthr)
        if (mark[(v - 1) >> 1]) mark[v] = 1;
      __syncthreads();
    }
    const int leaf0 = (1 << (n - 1)) - 1;
    uint32_t nbad_local = 0, first_good = 0xFFFFFFFFu;
    for (int w = tid; w < nw32; w += nthr) {
      uint32_t bits = 0;
      for (int l = 0; l < 32; ++l) {
        const int i = 32 * w + l;
        if (i < D && mark[leaf0 + (i >> 1)]) bits |= 1u << l;
      }
      badw[w] = bits;
      nbad_local += __popc(bits);
      const uint32_t valid = (32 * w + 32 <= D) ? 0xFFFFFFFFu : ((1u << (D - 32 * w)) - 1u);
      const uint32_t good = ~bits & valid;
      if (good && first_good == 0xFFFFFFFFu) first_good = 32 * w + (__ffs(good) - 1);
    }
    if (first_good != 0xFFFFFFFFu) atomicMin(&sbuf[8], first_good);
    uint32_t nbad;
    block_excl_scan_u32(nbad_local, sbuf, &nbad);
    __syncthreads();
    const uint32_t ref = sbuf[8];
    const int nw64 = (D + 63) >> 6;
    uint64_t *bb = rp->badbits + (size_t)tj * nw64;
    for (int w = tid; w < nw64; w += nthr) {
      const uint64_t lo = badw[2 * w];
      const uint64_t hi = (2 * w + 1 < nw32) ? badw[2 * w + 1] : 0;
      bb[w] = lo | (hi << 32);
    }
    // explicit addresses: every bad address plus the reference (pruned), in
    // ascending order; the full mode evolves every address.
    uint32_t nex;
    if (rp->mode == 1) {
      const int per = (nw32 + nthr - 1) / nthr;
      const int w0 = min(nw32, tid * per), w1 = min(nw32, w0 + per);
      uint32_t c = 0;
      for (int w = w0; w < w1; ++w) {
        uint32_t f = badw[w];
        if (ref != 0xFFFFFFFFu && (ref >> 5) == (uint32_t)w) f |= 1u << (ref & 31);
        c += __popc(f);
      }
      uint32_t tot;
      uint32_t o = block_excl_scan_u32(c, sbuf, &tot);
      uint16_t *xl = rp->xlist + (size_t)tj * D;
      for (int w = w0; w < w1; ++w) {
        uint32_t f = badw[w];
        if (ref != 0xFFFFFFFFu && (ref >> 5) == (uint32_t)w) f |= 1u << (ref & 31);
        while (f) {
          const int l = __ffs(f) - 1;
          f &= f - 1;
          xl[o++] = (uint16_t)(32 * w + l);
        }
      }
      nex = tot << kb;
    } else {
      nex = (uint32_t)D << kb;
    }
    if (tid == 0) {
      rp->nbad[tj] = nbad;
      rp->ref[tj] = ref;
      rp->nexpl[tj] = nex;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// k_order: trajectories sorted into descending buckets of explicit work
// (log2 buckets), for the longest-first persistent schedule.  Also resets the
// queue head.  One workgroup.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_order(const Run R_) {
  const Run *rp = &R_;
  __shared__ uint32_t hist[33];
  __shared__ uint32_t base[33];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const uint32_t nt = rp->ntraj;
  if (tid < 33) hist[tid] = 0;
  __syncthreads();
  for (uint32_t t = tid; t < nt; t += nthr) {
    const uint32_t e = rp->nexpl[t];
    const int bkt = 32 - __clz(e);  // 0..32, larger work -> larger bucket
    atomicAdd(&hist[bkt], 1u);
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t acc = 0;
    for (int b = 32; b >= 0; --b) {
      base[b] = acc;
      acc += hist[b];
    }
    rp->counter[0] = 0;
  }
  __syncthreads();
  for (uint32_t t = tid; t < nt; t += nthr) {
    const uint32_t e = rp->nexpl[t];
    const int bkt = 32 - __clz(e);
    const uint32_t o = atomicAdd(&base[bkt], 1u);
    rp->order[o] = t;
  }
}

// ---------------------------------------------------------------------------
// k_digest: FNV-1a 64 of each candidate list (4 little-endian bytes each).
// ---------------------------------------------------------------------------
__global__ void k_digest(const Run R_) {
  const Run *rp = &R_;
  const uint32_t tj = blockIdx.x * blockDim.x + threadIdx.x;
  if (tj >= rp->ntraj) return;
  const uint32_t nc = min(rp->ncand[tj], rp->cand_cap);
  const uint32_t *c = rp->cand + (size_t)tj * rp->cand_cap;
  uint64_t h = 0xcbf29ce484222325ull;
  for (uint32_t j = 0; j < nc; ++j) {
    uint32_t x = c[j];
    for (int b = 0; b < 4; ++b) {
      h ^= (x & 0xFFu);
      h *= 0x100000001b3ull;
      x >>= 8;
    }
  }
  rp->digest[tj] = h;
}

// ---------------------------------------------------------------------------
// k_evolve helpers: tier-1 components (live tokens on the component's path)
// ---------------------------------------------------------------------------

// Level of site q (0 = ground; 1 = excited / L; 2 = R) for a tier-1 component
// of address a with live data tokens `live`, after the gates of slice s.
template <int ENC>
__device__ __forceinline__ int t1_level(const Tables *__restrict__ tb, int s,
                                        uint32_t a, uint32_t live, uint32_t memw,
                                        uint32_t q) {
  const int n = tb->n;
  const uint32_t v = q >> 1, slot = q & 1u;
  const int l = layer_of(v);
  if ((a >> (n - l)) != v + 1 - (1u << l)) return 0;
  const uint32_t tk = tb->tok[s][l][slot];
  if (tk == NONE) return 0;
  if (tk < (uint32_t)n) {
    const uint32_t bit = (a >> (n - 1 - tk)) & 1u;
    if (ENC == QUBIT) return (int)bit;
    return slot == 0 ? (bit ? 2 : 1) : (int)bit;
  }
  const int b = (int)tk - n;
  if (ENC == QUBIT) return (int)((live >> b) & 1u);
  return (int)(((tb->dmask[s] & memw & live) >> b) & 1u);
}

// Number of excited sites of a tier-1 component after the gates of slice s.
template <int ENC>
__device__ __forceinline__ uint32_t t1_exc(const Tables *__restrict__ tb, int s,
                                           uint32_t a, uint32_t live,
                                           uint32_t memw) {
  if (ENC == QUBIT) return __popc(a & tb->amask[s]) + __popc(live & tb->dmask[s]);
  return tb->nrouter[s] + __popc(a & tb->amask[s]) +
         __popc(memw & live & tb->dmask[s]);
}

// Site of token tk (address token t < n, data token n + b) of address a at
// slice s, or -1 when outside the tree.
__device__ __forceinline__ int t1_site(const Tables *__restrict__ tb, int s,
                                       uint32_t a, int tk) {
  const uint8_t ps = tb->pos[s][tk];
  if (ps == NONE) return -1;
  const int l = ps >> 1, slot = ps & 1;
  const uint32_t v = (1u << l) - 1u + (a >> (tb->n - l));
  return (int)(2 * v + slot);
}

__device__ __forceinline__ bool cand_bm(const uint32_t *cbm, uint32_t q) {
  return (cbm[q >> 5] >> (q & 31)) & 1u;
}

__device__ __forceinline__ bool cand_list(const uint32_t *cdec, int nc,
                                          uint32_t q) {
  for (int j = 0; j < nc; ++j)
    if ((cdec[j] & 0xFFFFu) == q) return true;
  return false;
}

// Does some candidate of slice s hit the tier-1 component?  With few
// candidates the decoded list is scanned; otherwise every excited token
// position is looked up in the slice's candidate bitmap.
template <int ENC>
__device__ __forceinline__ bool t1_hit(const Tables *__restrict__ tb, int s,
                                       uint32_t a, uint32_t live, uint32_t memw,
                                       bool big, int nc, const uint32_t *cdec,
                                       const uint32_t *cbm) {
  const int n = tb->n;
  if (!big) {
    for (int j = 0; j < nc; ++j) {
      const uint32_t c = cdec[j];
      const uint32_t tk = (c >> 20) & 0xFFu;
      if (tk == NONE) continue;
      const int l = (c >> 16) & 15;
      const uint32_t q = c & 0xFFFFu;
      const uint32_t v = q >> 1;
      if ((a >> (n - l)) != v + 1 - (1u << l)) continue;
      if (tk < (uint32_t)n) {
        if (ENC == QUTRIT && (q & 1u) == 0) return true;  // stored router
        if ((a >> (n - 1 - tk)) & 1u) return true;
      } else {
        const int b = (int)tk - n;
        if (ENC == QUBIT) {
          if ((live >> b) & 1u) return true;
        } else if (((tb->dmask[s] & memw & live) >> b) & 1u) {
          return true;
        }
      }
    }
    return false;
  }
  for (int t = 0; t < n; ++t) {
    const bool abit = (a >> (n - 1 - t)) & 1u;
    const uint8_t ps = tb->pos[s][t];
    if (ps == NONE) continue;
    const bool router = (ps & 1) == 0;
    if (!(abit || (ENC == QUTRIT && router))) continue;
    const int q = t1_site(tb, s, a, t);
    if (cand_bm(cbm, (uint32_t)q)) return true;
  }
  const uint32_t dl = ENC == QUBIT ? (live & tb->dmask[s]) : (memw & live & tb->dmask[s]);
  for (int b = 0; b < tb->k; ++b) {
    if (!((dl >> b) & 1u)) continue;
    const int q = t1_site(tb, s, a, n + b);
    if (q >= 0 && cand_bm(cbm, (uint32_t)q)) return true;
  }
  return false;
}

// ---------------------------------------------------------------------------
// Tier-2 records (explicit site lists in the pool).
// ---------------------------------------------------------------------------
template <int ENC>
struct Rec {
  uint16_t *r;
  static constexpr uint32_t SM = ENC == QUTRIT ? 0x7FFFu : 0xFFFFu;
  __device__ __forceinline__ int cnt() const { return r[0]; }
  __device__ __forceinline__ uint32_t raw(int j) const { return r[2 + j]; }
  __device__ __forceinline__ uint32_t site(int j) const { return r[2 + j] & SM; }
  __device__ __forceinline__ int find_site(uint32_t q) const {
    const int c = r[0];
    for (int j = 0; j < c; ++j)
      if ((r[2 + j] & SM) == q) return j;
    return -1;
  }
  __device__ __forceinline__ int find_raw(uint32_t x) const {
    const int c = r[0];
    for (int j = 0; j < c; ++j)
      if (r[2 + j] == x) return j;
    return -1;
  }
  __device__ __forceinline__ void remove(int j) {
    const int c = r[0] - 1;
    r[2 + j] = r[2 + c];
    r[0] = (uint16_t)c;
  }
  __device__ __forceinline__ bool add(uint32_t x, int lmax) {
    const int c = r[0];
    if (c >= lmax) return false;
    r[2 + c] = (uint16_t)x;
    r[0] = (uint16_t)(c + 1);
    return true;
  }
  // routing direction of node v: qubit 0/1; qutrit -1 (W), 0 (L), 1 (R)
  __device__ __forceinline__ int dir(uint32_t v) const {
    const int j = find_site(2 * v);
    if (ENC == QUBIT) return j >= 0 ? 1 : 0;
    if (j < 0) return -1;
    return (r[2 + j] & LV_R_BIT) ? 1 : 0;
  }
};

// Apply the gates of slice s to a tier-2 record (App. A schedule, App. C
// gate set; qutrit circuit as in the oracle's conventions).
template <int ENC>
__device__ void t2_gates(const Tables *__restrict__ tb, int s, Rec<ENC> R,
                         uint32_t a, uint32_t &word, uint32_t *err) {
  const int n = tb->n, lmax = tb->lmax;
  const int ct = tb->copy_t[s];
  if (ct >= 0 && ((a >> (n - 1 - ct)) & 1u)) {
    const int j = R.find_site(1);
    if (j >= 0)
      R.remove(j);
    else if (!R.add(1, lmax))
      atomicOr(err, ERR_LIST);
  }
  const int sl = tb->store_l[s];
  if (sl >= 0) {
    if (ENC == QUBIT) {
      for (int j = 0; j < R.cnt(); ++j) {
        const uint32_t q = R.site(j);
        if (layer_of(q >> 1) == sl) R.r[2 + j] = (uint16_t)(q ^ 1u);
      }
    } else {
      // nodes of layer sl that a router of layer sl-1 points to (the root
      // for sl = 0) exchange (W,b) <-> (L_b, 0)
      uint32_t gated[4];
      int ng = 0;
      if (sl == 0) {
        gated[ng++] = 0;
      } else {
        for (int j = 0; j < R.cnt() && ng < 4; ++j) {
          const uint32_t x = R.raw(j), q = x & Rec<ENC>::SM;
          if (q & 1u) continue;
          const uint32_t v = q >> 1;
          if (layer_of(v) != sl - 1) continue;
          gated[ng++] = 2 * v + 1 + ((x & LV_R_BIT) ? 1u : 0u);
        }
      }
      for (int g = 0; g < ng; ++g) {
        const uint32_t v = gated[g];
        const int jr = R.find_site(2 * v);
        const int jd = R.find_site(2 * v + 1);
        if (jr < 0) {
          if (jd >= 0) {
            R.remove(jd);
            R.add(2 * v | LV_R_BIT, lmax);
          } else if (!R.add(2 * v, lmax)) {
            atomicOr(err, ERR_LIST);
          }
        } else if (jd < 0) {
          const bool isR = (R.raw(jr) & LV_R_BIT) != 0;
          R.remove(jr);
          if (isR) R.add(2 * v + 1, lmax);
        }
      }
    }
  }
  const uint32_t cm = tb->cswap[s];
  if (cm) {
    for (int j = 0; j < R.cnt(); ++j) {
      const uint32_t q = R.site(j);
      if (!(q & 1u)) continue;
      const uint32_t v = q >> 1;
      const int l = layer_of(v);
      if ((cm >> l) & 1u) {
        const int d = R.dir(v);
        if (d >= 0) R.r[2 + j] = (uint16_t)(2 * (2 * v + 1 + d) + 1);
      } else if (l >= 1 && ((cm >> (l - 1)) & 1u)) {
        const uint32_t p = (v - 1) >> 1;
        const int d = R.dir(p);
        if (d >= 0 && v == 2 * p + 1 + (uint32_t)d) R.r[2 + j] = (uint16_t)(2 * p + 1);
      }
    }
  }
  const int bb = tb->bus_b[s];
  if (bb >= 0) {
    const int j = R.find_site(1);
    const uint32_t bus = R.r[1];
    const bool bbit = (bus >> bb) & 1u;
    if (j >= 0 && !bbit) {
      R.remove(j);
      R.r[1] = (uint16_t)(bus | (1u << bb));
    } else if (j < 0 && bbit) {
      if (!R.add(1, lmax)) atomicOr(err, ERR_LIST);
      R.r[1] = (uint16_t)(bus & ~(1u << bb));
    }
  }
  const int fb = tb->fetch_b[s];
  if (fb >= 0) {
    const uint32_t v0 = (1u << (n - 1)) - 1u;
    if (ENC == QUBIT) {
      for (int j = 0; j < R.cnt(); ++j) {
        const uint32_t q = R.site(j);
        if (!(q & 1u) || (q >> 1) < v0) continue;
        const uint32_t v = q >> 1, p = v - v0;
        const uint32_t cell = 2 * p + (uint32_t)R.dir(v);
        if ((tb->mem[cell] >> fb) & 1u) word ^= W_SIGN;
      }
    } else {
      uint32_t leaf[4], lv[4];
      int nl = 0;
      for (int j = 0; j < R.cnt() && nl < 4; ++j) {
        const uint32_t x = R.raw(j), q = x & Rec<ENC>::SM;
        if ((q & 1u) || (q >> 1) < v0) continue;
        leaf[nl] = q >> 1;
        lv[nl++] = (x & LV_R_BIT) ? 1u : 0u;
      }
      for (int g = 0; g < nl; ++g) {
        const uint32_t v = leaf[g], p = v - v0;
        if ((tb->mem[2 * p + lv[g]] >> fb) & 1u) {
          const int jd = R.find_site(2 * v + 1);
          if (jd >= 0)
            R.remove(jd);
          else if (!R.add(2 * v + 1, lmax))
            atomicOr(err, ERR_LIST);
        }
      }
    }
  }
}

// Explicit site list of a tier-1 component at slice s (after the gates).
template <int ENC>
__device__ void t1_materialize(const Tables *__restrict__ tb, int s, uint32_t a,
                               uint32_t live, uint32_t memw, Rec<ENC> R,
                               uint32_t *err) {
  const int n = tb->n, k = tb->k, lmax = tb->lmax;
  R.r[0] = 0;
  uint32_t bus = 0;
  for (int t = 0; t < n; ++t) {
    const bool abit = (a >> (n - 1 - t)) & 1u;
    const int q = t1_site(tb, s, a, t);
    if (q < 0) continue;
    if (ENC == QUTRIT && (q & 1) == 0) {
      if (!R.add((uint32_t)q | (abit ? LV_R_BIT : 0u), lmax)) atomicOr(err, ERR_LIST);
    } else if (abit) {
      if (!R.add((uint32_t)q, lmax)) atomicOr(err, ERR_LIST);
    }
  }
  for (int b = 0; b < k; ++b) {
    const int q = t1_site(tb, s, a, n + b);
    if (ENC == QUBIT) {
      const bool lb = (live >> b) & 1u;
      if (q >= 0) {
        if (lb && !R.add((uint32_t)q, lmax)) atomicOr(err, ERR_LIST);
      } else if (lb) {
        bus |= 1u << b;  // not yet in, or already back on the bus
      }
    } else {
      const bool vb = ((memw & live) >> b) & 1u;
      if (q >= 0) {
        if (((tb->dmask[s] >> b) & 1u) && vb && !R.add((uint32_t)q, lmax))
          atomicOr(err, ERR_LIST);
      } else if (s >= 4 * n + 2 * b + 1 && vb) {
        bus |= 1u << b;  // fetched value already on the bus
      }
    }
  }
  R.r[1] = (uint16_t)bus;
}

// ---------------------------------------------------------------------------
// k_evolve
// ---------------------------------------------------------------------------
struct EvSmem {
  double *red;      // [2 * nw * 8]
  double *scanb;    // [nw]
  uint32_t *cstart; // [MAXT + 1]
  uint32_t *cdec;   // [NCS]
  uint32_t *Jb;     // [JMAX]
  int *misc;        // [8]
  uint32_t *cbm;    // [(M + 31) / 32]
  uint32_t *st;     // [e_cap] when the state lives in LDS
};

__host__ __device__ inline uint32_t align16(uint32_t x) { return (x + 15u) & ~15u; }

__host__ __device__ inline uint32_t evolve_fixed_bytes(int M, int threads) {
  const int nw = threads >> 6;
  uint32_t b = 0;
  b += align16(2 * nw * 8 * 8);
  b += align16(nw * 8);
  b += align16((MAXT + 1) * 4);
  b += align16(NCS * 4);
  b += align16(JMAX * 4);
  b += align16(8 * 4);
  b += align16(((M + 31) / 32) * 4);
  return b;
}

__device__ inline EvSmem carve(unsigned char *base, int M, int threads) {
  const int nw = threads >> 6;
  EvSmem m;
  unsigned char *p = base;
  m.red = reinterpret_cast<double *>(p);
  p += align16(2 * nw * 8 * 8);
  m.scanb = reinterpret_cast<double *>(p);
  p += align16(nw * 8);
  m.cstart = reinterpret_cast<uint32_t *>(p);
  p += align16((MAXT + 1) * 4);
  m.cdec = reinterpret_cast<uint32_t *>(p);
  p += align16(NCS * 4);
  m.Jb = reinterpret_cast<uint32_t *>(p);
  p += align16(JMAX * 4);
  m.misc = reinterpret_cast<int *>(p);
  p += align16(8 * 4);
  m.cbm = reinterpret_cast<uint32_t *>(p);
  p += align16(((M + 31) / 32) * 4);
  m.st = reinterpret_cast<uint32_t *>(p);
  return m;
}

template <int ENC, bool SL>
__global__ void __launch_bounds__(1024) k_evolve(const Tables *__restrict__ tb,
                                                 const Run R_) {
  const Run *rp = &R_;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int n = tb->n, T = tb->T, M = tb->M, D = tb->D, emax = tb->emax;
  const int kb = ENC == QUBIT ? tb->k : 0;
  const uint32_t K2m = ENC == QUBIT ? (uint32_t)tb->K2 - 1u : 0u;
  const uint32_t kmask = (1u << tb->k) - 1u;
  const double *__restrict__ wpow = tb->wpow + emax;
  const double *__restrict__ apow = tb->apow + emax;
  const uint32_t *__restrict__ mem = tb->mem;
  EvSmem sm = carve(smem, M, nthr);
  const uint32_t e_cap = rp->e_cap;
  uint32_t *st = SL ? sm.st : rp->gstate + (size_t)blockIdx.x * e_cap;
  uint16_t *pool = rp->pool + (size_t)blockIdx.x * tb->D * (ENC == QUBIT ? tb->K2 : 1) * tb->rec;
  const int rec = tb->rec;
  const bool pruned = rp->mode == 1;
  const uint32_t ccap = rp->cand_cap;
  int big_prev_s = 0, big_prev_cb = 0, big_prev_nc = 0;
  for (int w = tid; w < (M + 31) / 32; w += nthr) sm.cbm[w] = 0u;

  for (uint32_t iter = 0;; ++iter) {
    uint32_t qslot;
    __syncthreads();
    if (rp->persistent) {
      if (tid == 0) sm.misc[0] = (int)atomicAdd(rp->counter, 1u);
      __syncthreads();
      qslot = (uint32_t)sm.misc[0];
    } else {
      qslot = blockIdx.x + iter * gridDim.x;
    }
    if (qslot >= rp->ntraj) break;
    const uint32_t tj = rp->persistent ? rp->order[qslot] : qslot;
    const uint32_t traj = rp->traj0 + tj;
    const uint32_t E = rp->nexpl[tj];
    const uint32_t nct = min(rp->ncand[tj], ccap);
    const uint32_t *__restrict__ cand = rp->cand + (size_t)tj * ccap;
    const uint16_t *__restrict__ xl = pruned ? rp->xlist + (size_t)tj * D : nullptr;
    const uint32_t ref = rp->ref[tj];
    const uint64_t *__restrict__ bad = rp->badbits + (size_t)tj * ((D + 63) >> 6);
    const uint32_t spt = (E + nthr - 1) / nthr;

    // slice boundaries of the ascending candidate list
    for (uint32_t j = tid; j <= nct; j += nthr) {
      const int sj = j < nct ? (int)(cand[j] / (uint32_t)M) + 1 : T;
      const int sp = j > 0 ? (int)(cand[j - 1] / (uint32_t)M) + 1 : 0;
      for (int ss = sp + 1; ss <= sj; ++ss) sm.cstart[ss] = j;
    }
    if (tid == 0) sm.cstart[T + 0] = nct;
    // initial components: the data-loading input (after the first wall)
    for (uint32_t j = 0; j < spt; ++j) {
      const uint32_t slot = tid * spt + j;
      if (slot >= E) break;
      const uint32_t live = ENC == QUBIT ? (slot & K2m) : kmask;
      st[j * nthr + tid] = W_ALIVE | (live << W_LIVE_SH);
    }
    __syncthreads();

    bool ref_alive = pruned && ref != 0xFFFFFFFFu;
    int njumps = 0, first_jump = 0;
    uint32_t reft = 0;  // address bits of the reference
    if (ref != 0xFFFFFFFFu) reft = ref;

    for (int s = 1; s < T; ++s) {
      const uint32_t cb = sm.cstart[s];
      const int nc = (int)(sm.cstart[s + 1] - cb);
      const bool big = nc > NCS;
      if (nc > 0) {
        if (big) {
          if (big_prev_nc > 0) {  // clear the previous big slice's bits
            for (int j = tid; j < big_prev_nc; j += nthr) {
              const uint32_t q = cand[big_prev_cb + j] - (uint32_t)(big_prev_s - 1) * M;
              sm.cbm[q >> 5] = 0;
            }
            __syncthreads();
          }
          for (int j = tid; j < nc; j += nthr) {
            const uint32_t q = cand[cb + j] - (uint32_t)(s - 1) * M;
            atomicOr(&sm.cbm[q >> 5], 1u << (q & 31));
          }
          big_prev_s = s;
          big_prev_cb = (int)cb;
          big_prev_nc = nc;
        } else {
          for (int j = tid; j < nc; j += nthr) {
            const uint32_t q = cand[cb + j] - (uint32_t)(s - 1) * M;
            const uint32_t v = q >> 1;
            const int l = layer_of(v);
            const uint32_t tk = tb->tok[s][l][q & 1u];
            sm.cdec[j] = q | ((uint32_t)l << 16) | (tk << 20);
          }
        }
        __syncthreads();
      }

      // phase A: gates, K0 exposure (as if J were empty), hits and weights
      double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // hits, w_empty, w_hit, w_ref, R_good
      for (uint32_t j = 0; j < spt; ++j) {
        const uint32_t slot = tid * spt + j;
        if (slot >= E) break;
        uint32_t w = st[j * nthr + tid];
        if (!(w & W_ALIVE)) continue;
        const uint32_t a = xl ? xl[slot >> kb] : (slot >> kb);
        const uint32_t memw = ENC == QUTRIT ? mem[a] : 0u;
        const uint32_t e0 = w & W_E;
        uint32_t exc;
        bool hit = false;
        if (!(w & W_DEV)) {
          const uint32_t live = (w >> W_LIVE_SH) & 0xFFu;
          exc = t1_exc<ENC>(tb, s, a, live, memw);
          if (ENC == QUBIT) {
            const int fb = tb->fetch_b[s];
            if (fb >= 0 && ((live & mem[a]) >> fb) & 1u) w ^= W_SIGN;
          }
          if (nc > 0) hit = t1_hit<ENC>(tb, s, a, live, memw, big, nc, sm.cdec, sm.cbm);
        } else {
          Rec<ENC> R{pool + (size_t)slot * rec};
          t2_gates<ENC>(tb, s, R, a, w, rp->err);
          exc = R.cnt();
          if (nc > 0) {
            for (int q = 0; q < R.cnt() && !hit; ++q)
              hit = big ? cand_bm(sm.cbm, R.site(q)) : cand_list(sm.cdec, nc, R.site(q));
          }
        }
        if (nc > 0) {
          const double wt = wpow[e0];
          if (hit) {
            acc[0] += 1.0;
            acc[2] += wt;
          } else {
            acc[1] += wt;
          }
          if (a == ref) acc[3] += wt;
        }
        w = (w & ~W_E) | (e0 + exc);
        st[j * nthr + tid] = w;
      }
      if (nc == 0) continue;
      const double my_hit_w = acc[2];
      if (ref_alive) {
        // good branches other than the reference enter w(empty) through
        // their no-jump weights relative to the reference (Eq. maskweight)
        for (int i = tid; i < D; i += nthr) {
          if ((uint32_t)i == ref || ((bad[i >> 6] >> (i & 63)) & 1ull)) continue;
          int de = 0;
          for (int t = 0; t < n; ++t) {
            const int dt = (int)((i >> (n - 1 - t)) & 1) - (int)((reft >> (n - 1 - t)) & 1u);
            de += dt * (int)tb->cntA[s - 1][t];
          }
          if (ENC == QUTRIT) {
            const uint32_t mi = mem[i], mr = mem[reft];
            for (int b = 0; b < tb->k; ++b) {
              const int db = (int)((mi >> b) & 1u) - (int)((mr >> b) & 1u);
              de += db * (int)tb->cntD[s - 1][b];
            }
          }
          acc[4] += wpow[de];
        }
      }
      double* rbuf = sm.red + (s & 1) * (nthr >> 6) * 8;
      block_sum<5>(acc, rbuf);
      if (acc[0] == 0.0) continue;  // no component can jump: J is empty

      const double wgood = ref_alive ? acc[3] * acc[4] : 0.0;
      const double u = rp->forced ? rp->uaux[s] : uniform53(rp->seed, (uint32_t)s, 0, traj, 2u);
      const double w0 = acc[1] + wgood;
      const double r = u * (w0 + acc[2]);
      if (r < w0) continue;  // J empty: K0 already applied
      const double r2 = r - w0;

      // auxiliary component x*: components with empty masks form the first
      // block, the others follow in slot order (initial-label order)
      const double excl = block_excl_scan(my_hit_w, sm.scanb);
      if (tid == 0) sm.misc[1] = -1;
      __syncthreads();
      if (my_hit_w > 0.0 && excl <= r2) atomicMax(&sm.misc[1], tid);
      __syncthreads();
      if (sm.misc[1] == tid) {
        double cum = excl;
        int pick = -1, last = -1;
        for (uint32_t j = 0; j < spt; ++j) {
          const uint32_t slot = tid * spt + j;
          if (slot >= E) break;
          const uint32_t w = st[j * nthr + tid];
          if (!(w & W_ALIVE)) continue;
          const uint32_t a = xl ? xl[slot >> kb] : (slot >> kb);
          const uint32_t memw = ENC == QUTRIT ? mem[a] : 0u;
          bool hit = false;
          uint32_t exc;
          if (!(w & W_DEV)) {
            const uint32_t live = (w >> W_LIVE_SH) & 0xFFu;
            exc = t1_exc<ENC>(tb, s, a, live, memw);
            hit = t1_hit<ENC>(tb, s, a, live, memw, big, nc, sm.cdec, sm.cbm);
          } else {
            Rec<ENC> R{pool + (size_t)slot * rec};
            exc = R.cnt();
            for (int q = 0; q < R.cnt() && !hit; ++q)
              hit = big ? cand_bm(sm.cbm, R.site(q)) : cand_list(sm.cdec, nc, R.site(q));
          }
          if (!hit) continue;
          last = (int)j;
          cum += wpow[(w & W_E) - exc];
          if (cum > r2) {
            pick = (int)j;
            break;
          }
        }
        if (pick < 0) pick = last;
        // J = candidates of slice s among x*'s excited sites, with levels
        int nJ = 0;
        const uint32_t slot = tid * spt + (uint32_t)pick;
        const uint32_t w = st[pick * nthr + tid];
        const uint32_t a = xl ? xl[slot >> kb] : (slot >> kb);
        const uint32_t memw = ENC == QUTRIT ? mem[a] : 0u;
        if (!(w & W_DEV)) {
          const uint32_t live = (w >> W_LIVE_SH) & 0xFFu;
          if (!big) {
            for (int c = 0; c < nc; ++c) {
              const uint32_t q = sm.cdec[c] & 0xFFFFu;
              const int lev = t1_level<ENC>(tb, s, a, live, memw, q);
              if (lev && nJ < JMAX) sm.Jb[nJ++] = q | ((uint32_t)lev << 16);
            }
          } else {
            for (int tk = 0; tk < n + tb->k; ++tk) {
              const int q = t1_site(tb, s, a, tk);
              if (q < 0 || !cand_bm(sm.cbm, (uint32_t)q)) continue;
              const int lev = t1_level<ENC>(tb, s, a, live, memw, (uint32_t)q);
              if (lev && nJ < JMAX) sm.Jb[nJ++] = (uint32_t)q | ((uint32_t)lev << 16);
            }
          }
        } else {
          Rec<ENC> R{pool + (size_t)slot * rec};
          for (int c = 0; c < R.cnt(); ++c) {
            const uint32_t x = R.raw(c), q = x & Rec<ENC>::SM;
            const bool isc = big ? cand_bm(sm.cbm, q) : cand_list(sm.cdec, nc, q);
            if (!isc) continue;
            const uint32_t lev = (ENC == QUTRIT && (x & LV_R_BIT)) ? 2u : 1u;
            if (nJ < JMAX) sm.Jb[nJ++] = q | (lev << 16);
          }
        }
        sm.misc[2] = nJ;
      }
      __syncthreads();
      const int nJ = sm.misc[2];

      // phase C: K_J on every component (survivors keep J's sites excited)
      for (uint32_t j = 0; j < spt; ++j) {
        const uint32_t slot = tid * spt + j;
        if (slot >= E) break;
        uint32_t w = st[j * nthr + tid];
        if (!(w & W_ALIVE)) continue;
        const uint32_t a = xl ? xl[slot >> kb] : (slot >> kb);
        const uint32_t memw = ENC == QUTRIT ? mem[a] : 0u;
        if (!(w & W_DEV)) {
          uint32_t live = (w >> W_LIVE_SH) & 0xFFu;
          bool ok = true, dev = false;
          for (int c = 0; c < nJ && ok; ++c) {
            const uint32_t x = sm.Jb[c], q = x & 0xFFFFu;
            ok = t1_level<ENC>(tb, s, a, live, memw, q) == (int)(x >> 16);
          }
          if (!ok) {
            st[j * nthr + tid] = 0u;
            continue;
          }
          uint32_t kill = 0;
          for (int c = 0; c < nJ; ++c) {
            const uint32_t q = sm.Jb[c] & 0xFFFFu;
            const uint32_t v = q >> 1;
            const int l = layer_of(v);
            const uint32_t tk = tb->tok[s][l][q & 1u];
            if (tk < (uint32_t)n)
              dev = true;
            else
              kill |= 1u << (tk - (uint32_t)n);
          }
          if (dev) {
            Rec<ENC> R{pool + (size_t)slot * rec};
            t1_materialize<ENC>(tb, s, a, live, memw, R, rp->err);
            for (int c = 0; c < nJ; ++c) {
              const uint32_t x = sm.Jb[c], q = x & 0xFFFFu;
              const uint32_t raw = (ENC == QUTRIT && (x >> 16) == 2u) ? (q | LV_R_BIT) : q;
              const int jj = R.find_raw(raw);
              if (jj >= 0) R.remove(jj);
            }
            w |= W_DEV;
          }
          live &= ~kill;
          w = (w & ~(0xFFu << W_LIVE_SH)) | (live << W_LIVE_SH);
        } else {
          Rec<ENC> R{pool + (size_t)slot * rec};
          bool ok = true;
          for (int c = 0; c < nJ && ok; ++c) {
            const uint32_t x = sm.Jb[c], q = x & 0xFFFFu;
            const uint32_t raw = (ENC == QUTRIT && (x >> 16) == 2u) ? (q | LV_R_BIT) : q;
            const int jj = R.find_raw(raw);
            if (jj < 0)
              ok = false;
            else
              R.remove(jj);
          }
          if (!ok) {
            st[j * nthr + tid] = 0u;
            continue;
          }
        }
        w = (w & ~W_E) | ((w & W_E) - (uint32_t)nJ);
        st[j * nthr + tid] = w;
      }
      ref_alive = false;  // a good branch never carries a candidate site
      ++njumps;
      if (!first_jump) first_jump = s;
    }

    if (big_prev_nc > 0) {  // leave the candidate bitmap clean for the next trajectory
      for (int j = tid; j < big_prev_nc; j += nthr) {
        const uint32_t q = cand[big_prev_cb + j] - (uint32_t)(big_prev_s - 1) * M;
        sm.cbm[q >> 5] = 0;
      }
      big_prev_nc = 0;
    }

    // second wall, tree measurement and fidelity (Alg. 1 steps 4-6)
    double fin[7] = {0, 0, 0, 0, 0, 0, 0};  // ov, w_ground, w_total, ov_ref, w_ref, G_a, G_w
    for (uint32_t j = 0; j < spt; ++j) {
      const uint32_t slot = tid * spt + j;
      if (slot >= E) break;
      const uint32_t w = st[j * nthr + tid];
      if (!(w & W_ALIVE)) continue;
      const uint32_t a = xl ? xl[slot >> kb] : (slot >> kb);
      const uint32_t e = w & W_E;
      const double wt = wpow[e];
      bool ground;
      uint32_t bus;
      if (!(w & W_DEV)) {
        const uint32_t live = (w >> W_LIVE_SH) & 0xFFu;
        ground = true;
        bus = ENC == QUBIT ? live : (mem[a] & live);
      } else {
        Rec<ENC> R{pool + (size_t)slot * rec};
        ground = R.cnt() == 0;
        bus = R.r[1];
      }
      fin[2] += wt;
      if (!ground) continue;
      fin[1] += wt;
      double term;
      if (ENC == QUBIT) {
        const bool neg = ((w & W_SIGN) != 0) ^ (bool)(__popc(bus & mem[a] & kmask) & 1);
        term = neg ? -apow[e] : apow[e];
      } else {
        term = bus == (mem[a] & kmask) ? apow[e] : 0.0;
      }
      fin[0] += term;
      if (a == ref) {
        fin[3] += term;
        fin[4] += wt;
      }
    }
    if (ref_alive) {
      for (int i = tid; i < D; i += nthr) {
        if ((uint32_t)i == ref || ((bad[i >> 6] >> (i & 63)) & 1ull)) continue;
        int de = 0;
        for (int t = 0; t < n; ++t) {
          const int dt = (int)((i >> (n - 1 - t)) & 1) - (int)((reft >> (n - 1 - t)) & 1u);
          de += dt * (int)tb->cntA[T - 1][t];
        }
        if (ENC == QUTRIT) {
          const uint32_t mi = mem[i], mr = mem[reft];
          for (int b = 0; b < tb->k; ++b) {
            const int db = (int)((mi >> b) & 1u) - (int)((mr >> b) & 1u);
            de += db * (int)tb->cntD[T - 1][b];
          }
        }
        fin[5] += apow[de];
        fin[6] += wpow[de];
      }
    }
    __syncthreads();
    block_sum<7>(fin, sm.red);
    if (tid == 0) {
      double ov = fin[0], wg = fin[1], wt = fin[2];
      if (ref_alive) {  // XOR mirror / scalar prediction of the good groups
        ov += fin[3] * fin[5];
        wg += fin[4] * fin[6];
        wt += fin[4] * fin[6];
      }
      const double uf = rp->forced ? rp->ufin : uniform53(rp->seed, 0, 0, traj, 3u);
      const bool qg = uf * wt < wg;
      const double norm = 1.0 / ((double)D * (double)(ENC == QUBIT ? tb->K2 : 1));
      rp->fid[tj] = (qg && wg > 0.0) ? ov * ov / wg * norm : 0.0;
      if (rp->st) {
        qram_traj_stats o;
        o.n_cand = rp->ncand[tj];
        o.n_bad = rp->nbad[tj];
        o.ref_addr = ref;
        o.n_explicit = E;
        o.n_jumps = (uint16_t)njumps;
        o.first_jump_slice = (uint16_t)first_jump;
        o.ref_survived = (uint8_t)(ref != 0xFFFFFFFFu && njumps == 0);
        o.q_ground = (uint8_t)qg;
        o.flags = (uint8_t)((rp->ncand[tj] > ccap ? 1 : 0));
        o.pad = 0;
        o.fid_pre = wt > 0.0 ? ov * ov / wt * norm : 0.0;
        rp->st[tj] = o;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_sample(const Tables *tb, const Run &rp, uint32_t ntraj,
                         uint32_t grid, hipStream_t s) {
  (void)ntraj;
  hipLaunchKernelGGL(k_sample, dim3(grid), dim3(256), 0, s, tb, rp);
  return hipGetLastError();
}

hipError_t launch_classify(const Tables *tb, const Run &rp, uint32_t ntraj,
                           uint32_t grid, int D, hipStream_t s) {
  (void)ntraj;
  const size_t lds = (size_t)((D + 31) / 32) * 4 + 16 * 4 + (size_t)D;
  hipLaunchKernelGGL(k_classify, dim3(grid), dim3(256), lds, s, tb, rp);
  return hipGetLastError();
}

hipError_t launch_order(const Tables *tb, const Run &rp, uint32_t ntraj,
                        hipStream_t s) {
  (void)tb;
  (void)ntraj;
  hipLaunchKernelGGL(k_order, dim3(1), dim3(1024), 0, s, rp);
  return hipGetLastError();
}

hipError_t launch_digest(const Run &rp, uint32_t ntraj, hipStream_t s) {
  hipLaunchKernelGGL(k_digest, dim3((ntraj + 255) / 256), dim3(256), 0, s, rp);
  return hipGetLastError();
}

uint32_t evolve_lds_bytes(int n, int T, int M, int threads, uint32_t e_cap,
                          bool state_lds) {
  (void)n;
  (void)T;
  return evolve_fixed_bytes(M, threads) + (state_lds ? e_cap * 4u : 0u);
}

hipError_t evolve_prepare(int lds_max) {
  hipError_t e = hipSuccess;
  const void *fns[4] = {reinterpret_cast<const void *>(&k_evolve<QUBIT, true>),
                        reinterpret_cast<const void *>(&k_evolve<QUBIT, false>),
                        reinterpret_cast<const void *>(&k_evolve<QUTRIT, true>),
                        reinterpret_cast<const void *>(&k_evolve<QUTRIT, false>)};
  for (const void *f : fns) {
    const hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
    if (r != hipSuccess) e = r;
  }
  return e;
}

hipError_t launch_evolve(const Tables *tb, const Run &rp, int enc,
                         uint32_t grid, int threads, uint32_t lds_bytes,
                         bool state_lds, hipStream_t s) {
  if (enc == QUBIT) {
    if (state_lds)
      hipLaunchKernelGGL((k_evolve<QUBIT, true>), dim3(grid), dim3(threads), lds_bytes, s, tb, rp);
    else
      hipLaunchKernelGGL((k_evolve<QUBIT, false>), dim3(grid), dim3(threads), lds_bytes, s, tb, rp);
  } else {
    if (state_lds)
      hipLaunchKernelGGL((k_evolve<QUTRIT, true>), dim3(grid), dim3(threads), lds_bytes, s, tb, rp);
    else
      hipLaunchKernelGGL((k_evolve<QUTRIT, false>), dim3(grid), dim3(threads), lds_bytes, s, tb, rp);
  }
  return hipGetLastError();
}

}  // namespace qr

namespace qr {

int evolve_occupancy(int enc, bool state_lds, int threads, uint32_t lds_bytes) {
  int blocks = 0;
  hipError_t e;
  if (enc == QUBIT)
    e = state_lds ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_evolve<QUBIT, true>, threads, lds_bytes)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_evolve<QUBIT, false>, threads, lds_bytes);
  else
    e = state_lds ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_evolve<QUTRIT, true>, threads, lds_bytes)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_evolve<QUTRIT, false>, threads, lds_bytes);
  if (e != hipSuccess) return 0;
  return blocks;
}

}  // namespace qr
