// HIP kernels (gfx950) of the damped bucket-brigade QRAM trajectory simulator:
// candidate sampling, branch classification, work bucketing and candidate
// digests.  The evolution kernel lives in qram_evolve.hip.
//
//   k_sample    candidate history of each trajectory (Sec. IV D, first step of
//               the joint sampler): i.i.d. Bernoulli(gamma) site-slices drawn by
//               a geometric walk over 64-site blocks, Philox4x32-10 counters.
//   k_classify  bad-address set of the marking rule (Eq. subtree / Eq.
//               badrange, or Eq. subtree for qubit damping candidates on
//               request), reference = smallest good address, and the
//               ascending list of explicitly evolved addresses (Alg. 1 steps
//               1-2).
//   k_order     groups trajectories into buckets of explicit work, longest
//               first inside each bucket, and resets the queue heads.
//   k_sample_depol  depolarizing faults (Sec. II B, placement of App. C):
//               Bernoulli(eps) on the active positions of each slice, the
//               same geometric walk with its own counters (tag 4), the type
//               from the third word of the same Philox draw.
#include "qram_device.h"

namespace qr {

// ---------------------------------------------------------------------------
// k_sample
// ---------------------------------------------------------------------------
// MODE 0 counts the candidates of block b, 1 also writes them to out[base..]
// (below cap), 2 keeps the first four of the thread in buf (cnt counts on
// from its value on entry).
template <int MODE>
__device__ __forceinline__ uint32_t walk_block(uint32_t b, uint32_t len,
                                               uint32_t traj, uint32_t k0,
                                               uint32_t k1, const uint64_t *G,
                                               uint32_t *out, uint32_t base,
                                               uint32_t cap, uint32_t (&buf)[4],
                                               uint32_t cnt = 0) {
  uint32_t pos = 0;
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
    const uint32_t L = 64u * b + pos + lo;
    if (MODE == 1 && base + cnt < cap) out[base + cnt] = L;
    if (MODE == 2) {
      buf[0] = cnt == 0 ? L : buf[0];
      buf[1] = cnt == 1 ? L : buf[1];
      buf[2] = cnt == 2 ? L : buf[2];
      buf[3] = cnt == 3 ? L : buf[3];
    }
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
    // one walk keeps each thread's first four candidates in registers; a
    // second walk writes them only when some thread of the block had more
    uint32_t cnt = 0, buf[4] = {0, 0, 0, 0};
    for (uint32_t b = b0; b < b1; ++b) {
      const uint32_t len = (uint32_t)min((uint64_t)64, S - 64ull * b);
      cnt = walk_block<2>(b, len, traj, k0, k1, G, nullptr, 0, 0, buf, cnt);
    }
    uint32_t total;
    const uint32_t off = block_excl_scan_u32(cnt, sbuf, &total);
    uint32_t *out = rp->cand + (size_t)tj * cap;
    if (__syncthreads_or(cnt > 4u)) {
      if (cnt) {
        uint32_t o = off;
        for (uint32_t b = b0; b < b1; ++b) {
          const uint32_t len = (uint32_t)min((uint64_t)64, S - 64ull * b);
          o += walk_block<1>(b, len, traj, k0, k1, G, out, o, cap, buf);
        }
      }
    } else {
#pragma unroll
      for (uint32_t i = 0; i < 4; ++i)
        if (i < cnt && off + i < cap) out[off + i] = buf[i];
    }
    if (tid == 0) {
      rp->ncand[tj] = total;
      if (total > cap) atomicOr(rp->err, ERR_CAND);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// k_sample_depol
// ---------------------------------------------------------------------------
// Fault types: qubits and the qutrit data slot take X, Z or ZX (index
// (w2 * 3) >> 32), a qutrit router one of the eight nontrivial Weyl
// operators Z^b X^a (index (w2 * 8) >> 32); stored as a | b << 2.
__device__ __forceinline__ uint32_t depol_type(bool router3, uint32_t w2) {
  if (!router3) {
    const uint32_t i = (uint32_t)(((uint64_t)w2 * 3u) >> 32);
    return i == 0 ? 1u : (i == 1 ? 4u : 5u);  // X, Z, ZX
  }
  const uint32_t i = (uint32_t)(((uint64_t)w2 * 8u) >> 32);
  const uint32_t a = (i + 1) / 3, b = (i + 1) % 3;  // (0,1) (0,2) (1,0) ... (2,2)
  return a | (b << 2);
}

// Walk block b of the depolarizing index space; MODE 0 counts, 1 writes.
template <int MODE>
__device__ __forceinline__ uint32_t walk_block_dep(const Tables *__restrict__ tb, uint32_t b, uint32_t len,
                                                   uint32_t traj, uint32_t k0, uint32_t k1, const uint64_t *G,
                                                   uint32_t *out, uint32_t base, uint32_t cap) {
  uint32_t pos = 0, cnt = 0;
  int s = 1;
  for (uint32_t j = 0;; ++j) {
    const uint4 w = philox10(make_uint4(b, j, traj, 4u), k0, k1);
    const uint64_t u = (uint64_t)w.x | ((uint64_t)w.y << 32);
    const uint32_t rem = len - pos;
    if (!(u < G[rem - 1])) break;
    uint32_t lo = 0, hi = rem - 1;
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (u < G[mid])
        hi = mid;
      else
        lo = mid + 1;
    }
    const uint32_t L = 64u * b + pos + lo;
    if (MODE == 1 && base + cnt < cap) {
      while (tb->dep_off[s + 1] <= L) ++s;
      const uint32_t q = L - tb->dep_off[s];
      const bool router3 = tb->enc == QUTRIT && (q & 1u) == 0;
      out[base + cnt] = q | ((uint32_t)s << 16) | (depol_type(router3, w.z) << 24);
    }
    ++cnt;
    pos += lo + 1;
    if (pos >= len) break;
  }
  return cnt;
}

__global__ void __launch_bounds__(256) k_sample_depol(const Tables *__restrict__ tb, const Run R_) {
  const Run *rp = &R_;
  __shared__ uint64_t G[64];
  __shared__ uint32_t sbuf[16];
  const int tid = threadIdx.x, nthr = blockDim.x;
  if (tid < 64) G[tid] = tb->Gp[tid];
  __syncthreads();
  const uint32_t S = tb->dep_off[tb->T];
  const uint32_t nb = (S + 63) / 64;
  const uint32_t per = (nb + nthr - 1) / nthr;
  const uint32_t b0 = min(nb, tid * per), b1 = min(nb, b0 + per);
  const uint32_t k0 = (uint32_t)rp->seed, k1 = (uint32_t)(rp->seed >> 32);
  const uint32_t cap = rp->dep_cap;
  for (uint32_t tj = blockIdx.x; tj < rp->ntraj; tj += gridDim.x) {
    const uint32_t traj = rp->traj0 + tj;
    uint32_t cnt = 0;
    for (uint32_t b = b0; b < b1; ++b)
      cnt += walk_block_dep<0>(tb, b, min(64u, S - 64u * b), traj, k0, k1, G, nullptr, 0, 0);
    uint32_t total;
    const uint32_t off = block_excl_scan_u32(cnt, sbuf, &total);
    uint32_t *out = rp->dep + (size_t)tj * cap;
    if (cnt) {
      uint32_t o = off;
      for (uint32_t b = b0; b < b1; ++b)
        o += walk_block_dep<1>(tb, b, min(64u, S - 64u * b), traj, k0, k1, G, out, o, cap);
    }
    if (tid == 0) {
      rp->ndep[tj] = total;
      if (total > cap) atomicOr(rp->err, ERR_DEP);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// k_classify: marks the range node of every candidate, propagates marks down
// the tree, and derives the bad bitmap, the reference and the explicit list.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t range_node(int enc, bool subtree, uint32_t v) {
  // Eq. subtree: the qutrit encoding, and the qubit encoding when the
  // damping-only subtree marking is chosen (damping creates no strays)
  if (enc == QUTRIT || subtree) return v;
  // Eq. badrange: a left child below the root's children inherits its
  // parent's range; right children and the root's children mark their own
  // subtree; the root marks everything.
  while (v > 2 && (v & 1u)) v = (v - 1) >> 1;
  return v;
}

__global__ void __launch_bounds__(256) k_classify(const Tables *__restrict__ tb,
                                                  const Run R_, uint32_t subtree) {
  const Run *rp = &R_;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int n = tb->n, D = tb->D, M = tb->M, enc = tb->enc;
  const int nw32 = (D + 31) >> 5;
  uint32_t *badw = reinterpret_cast<uint32_t *>(smem);  // [nw32]
  uint32_t *sbuf = badw + nw32;                         // [16]
  uint32_t *wpos = sbuf + 16;                           // [nw32]
  uint8_t *mark = reinterpret_cast<uint8_t *>(wpos + nw32);  // [D - 1]
  const uint32_t cap = rp->cand_cap;
  const int kb = __ffs(tb->K2) - 1;  // components per address = 2^kb
  for (uint32_t tj = blockIdx.x; tj < rp->ntraj; tj += gridDim.x) {
    for (int v = tid; v < D - 1; v += nthr) mark[v] = 0;
    if (tid == 0) sbuf[8] = 0xFFFFFFFFu;
    __syncthreads();
    const uint32_t nc = min(rp->ncand[tj], cap);
    const uint32_t *cand = rp->cand + (size_t)tj * cap;
    for (uint32_t j = tid; j < nc; j += nthr) {
      const uint32_t q = cand[j] % (uint32_t)M;
      mark[range_node(enc, subtree != 0, q >> 1)] = 1;
    }
    if (rp->dep) {  // depolarizing faults: the encoding's rule whatever their type
      const uint32_t nd = min(rp->ndep[tj], rp->dep_cap);
      const uint32_t *dp = rp->dep + (size_t)tj * rp->dep_cap;
      for (uint32_t j = tid; j < nd; j += nthr) mark[range_node(enc, false, (dp[j] & 0xFFFFu) >> 1)] = 1;
    }
    __syncthreads();
    // address i is bad when a node on its path, root to its leaf node, is
    // marked; one ballot per wave gives 64 addresses of the bad bitmap
    const int leaf0 = (1 << (n - 1)) - 1;
    const int nw64 = (D + 63) >> 6;
    uint64_t *bb = rp->badbits + (size_t)tj * nw64;
    uint32_t nbad_local = 0, first_good = 0xFFFFFFFFu;
    for (int base = 0; base < D; base += nthr) {
      const int i = base + tid;
      bool bad = false, present = i < D;
      if (i < D) {
        uint32_t v = (uint32_t)(leaf0 + (i >> 1));
        for (int l = 0; l < n; ++l) {  // n nodes: the leaf node up to the root
          bad |= mark[v] != 0;
          v = (v - 1) >> 1;
        }
        if (tb->aflag)  // pair input: the reference holds one bus word
          present = (tb->aflag[i] & 2u) != 0;
        else if (tb->cin)
          present = tb->cin[2 * i] != 0.0 || tb->cin[2 * i + 1] != 0.0;
      }
      const uint64_t m = __ballot(bad);
      const uint64_t pm = __ballot(present);  // the reference must be in the input
      const int word = (base >> 6) + (tid >> 6);
      if ((tid & 63) == 0 && word < nw64) {
        const int nv = min(64, D - 64 * word);
        const uint64_t valid = nv >= 64 ? ~0ull : ((1ull << nv) - 1ull);
        bb[word] = m & valid;
        badw[2 * word] = (uint32_t)(m & valid);
        if (2 * word + 1 < nw32) badw[2 * word + 1] = (uint32_t)((m & valid) >> 32);
        nbad_local += (uint32_t)__popcll(m & valid);
        const uint64_t good = ~m & valid & pm;
        if (good) first_good = min(first_good, (uint32_t)(64 * word + __ffsll((unsigned long long)good) - 1));
      }
    }
    if (first_good != 0xFFFFFFFFu) atomicMin(&sbuf[8], first_good);
    uint32_t nbad;
    block_excl_scan_u32(nbad_local, sbuf, &nbad);
    __syncthreads();
    const uint32_t ref = sbuf[8];
    // explicit addresses: every bad address plus the reference (pruned), in
    // ascending order; the full mode evolves every address.
    uint32_t nex;
    if (rp->mode == 1) {
      const int per = (nw32 + nthr - 1) / nthr;
      const int w0 = min(nw32, tid * per), w1 = min(nw32, w0 + per);
      uint32_t c = 0;
      // without a reference nothing can be predicted: with a pair input a
      // good address may hold several bus words, so every address is explicit
      const bool all = ref == 0xFFFFFFFFu && tb->aflag;
      const uint32_t vlast = (D & 31) ? ((1u << (D & 31)) - 1u) : 0xFFFFFFFFu;
      auto expl = [&](int w) -> uint32_t {
        if (all) return w == nw32 - 1 ? vlast : 0xFFFFFFFFu;
        uint32_t f = badw[w];
        if (ref != 0xFFFFFFFFu && (ref >> 5) == (uint32_t)w) f |= 1u << (ref & 31);
        return f;
      };
      for (int w = w0; w < w1; ++w) c += __popc(expl(w));
      uint32_t tot;
      uint32_t o = block_excl_scan_u32(c, sbuf, &tot);
      // first list position of each bitmap word; then every address writes
      // its own entry (position = its word's offset + the set bits below it)
      for (int w = w0; w < w1; ++w) {
        wpos[w] = o;
        o += __popc(expl(w));
      }
      __syncthreads();
      uint16_t *xl = rp->xlist + (size_t)tj * D;
      for (int i = tid; i < D; i += nthr) {
        const int w = i >> 5;
        const uint32_t f = expl(w);
        const uint32_t below = f & ((1u << (i & 31)) - 1u);
        if ((f >> (i & 31)) & 1u) xl[wpos[w] + (uint32_t)__popc(below)] = (uint16_t)i;
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
// k_order: bucket b admits trajectories with at most bkt_emax[b] explicit
// components; inside a bucket trajectories are ordered by decreasing log2 of
// their work.  In a split run the trajectories that drew a depolarizing
// fault go to a segment of their own after every bucket, [bucket_base[MAXB],
// bucket_base[MAXB + 1]), also longest first, which the plain engine takes.
// One workgroup.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_order(const Run R_) {
  const Run *rp = &R_;
  constexpr int NF = 33;  // log2 bins inside a bucket
  constexpr int XF = MAXB * NF;  // the split run's plain-engine bins: XF .. XF + NF - 1
  __shared__ uint32_t hist[XF + NF];
  __shared__ uint32_t base[XF + NF];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const uint32_t nt = rp->ntraj;
  const uint32_t nb = rp->nbkt;
  const bool split = rp->dsplit != 0;
  for (int i = tid; i < XF + NF; i += nthr) hist[i] = 0;
  __syncthreads();
  auto key = [&](uint32_t t) -> int {
    const uint32_t e = rp->nexpl[t];
    const int f = 32 - __clz(e);  // larger work -> earlier
    if (split && rp->ndep[t] != 0) return XF + (NF - 1 - f);
    uint32_t b = 0;
    while (b + 1 < nb && e > rp->bkt_emax[b]) ++b;
    return (int)b * NF + (NF - 1 - f);
  };
  for (uint32_t t = tid; t < nt; t += nthr) atomicAdd(&hist[key(t)], 1u);
  __syncthreads();
  if (tid == 0) {
    uint32_t acc = 0;
    for (uint32_t b = 0; b < (uint32_t)MAXB; ++b) {
      rp->bucket_base[b] = acc;
      for (int f = 0; f < NF; ++f) {
        base[b * NF + f] = acc;
        acc += hist[b * NF + f];
      }
      rp->counter[b] = 0;
    }
    rp->bucket_base[MAXB] = acc;
    for (int f = 0; f < NF; ++f) {
      base[XF + f] = acc;
      acc += hist[XF + f];
    }
    if (split) rp->bucket_base[MAXB + 1] = acc;
  }
  __syncthreads();
  for (uint32_t t = tid; t < nt; t += nthr) {
    const uint32_t o = atomicAdd(&base[key(t)], 1u);
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
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_sample(const Tables *tb, const Run &rp, uint32_t ntraj,
                         uint32_t grid, hipStream_t s) {
  (void)ntraj;
  hipLaunchKernelGGL(k_sample, dim3(grid), dim3(256), 0, s, tb, rp);
  return hipGetLastError();
}

hipError_t launch_classify(const Tables *tb, const Run &rp, uint32_t ntraj,
                           uint32_t grid, int D, bool subtree, hipStream_t s) {
  (void)ntraj;
  const size_t lds = (size_t)((D + 31) / 32) * 8 + 16 * 4 + (size_t)D;
  hipLaunchKernelGGL(k_classify, dim3(grid), dim3(256), lds, s, tb, rp, subtree ? 1u : 0u);
  return hipGetLastError();
}

hipError_t launch_sample_depol(const Tables *tb, const Run &rp, uint32_t grid, hipStream_t s) {
  hipLaunchKernelGGL(k_sample_depol, dim3(grid), dim3(256), 0, s, tb, rp);
  return hipGetLastError();
}

hipError_t launch_order(const Tables *tb, const Run &rp, hipStream_t s) {
  (void)tb;
  hipLaunchKernelGGL(k_order, dim3(1), dim3(1024), 0, s, rp);
  return hipGetLastError();
}

// Fill n words with v: clears flags and counters without a memset node, so
// the enqueued work can sit inside a caller's graph capture.
__global__ void k_fill_u32(uint32_t *p, uint32_t v, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, uint32_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3((n + 255) / 256), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_digest(const Run &rp, uint32_t ntraj, hipStream_t s) {
  hipLaunchKernelGGL(k_digest, dim3((ntraj + 255) / 256), dim3(256), 0, s, rp);
  return hipGetLastError();
}

}  // namespace qr
