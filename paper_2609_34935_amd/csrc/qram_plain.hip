// Plain full evolution (gfx950): the comparator of the pruned simulator.
// One workgroup per trajectory carries every component of every branch
// through the T-1 slices of the schedule, each with its own explicit list of
// excited tree sites and its own complex FP64 amplitude:
//   - each slice applies the schedule's gates to every component's list
//     (the bucket-brigade schedule of Sec. II A, the gate set of App. C),
//   - then one joint damping layer (Eq. layerkraus, Theorem 4): the
//     components hit by a candidate of the slice are weighed (Eq.
//     maskweight), one auxiliary draw picks x*, J = C_s cap X(x*), and K_J
//     multiplies every survivor by sqrt(gamma)^|J| a^(|X|-|J|),
//   - at the end the second Hadamard wall (qubit encoding), the tree
//     measurement and the fidelity with the ideal output (App. C).
// Nothing is predicted: no closed-form no-jump walk, no implicit components,
// no closed-form finalize.  Same random numbers as the other modes, so the
// same history, jumps and fidelity up to rounding.
#include "qram_device.h"

namespace qr {
namespace {

constexpr int PL_GATED = 16;  // gated nodes of one qutrit store / fetch at most

// Explicit site list of one component in the workgroup's pool: [0] count
// (PL_DEAD once annihilated), [1] bus word, [2] exposure e, [3] phase
// index, [4 ..] sites.  In the pool the words of a record sit in pieces of
// eight (16 bytes): piece p of component y at word (p E + y) 8 of the
// trajectory's E components, so the threads of a wave, which work on
// consecutive components, read and write each piece as one contiguous
// run; a slab in shared memory holds a record contiguously. a qutrit router site carries its level in bit 15
// (set: R, clear: L).  The component's amplitude is the stored complex
// number times a^e times (-1)^(ph & 1) w3^(ph >> 1): the damping factors
// a^|X| of the slices and the phases of the gates and faults are counted
// in the record and multiplied in where an amplitude is needed (the draw's
// weights, a jump, the final sums), so that a slice without a jump does
// not touch the amplitude.
constexpr uint16_t PL_DEAD = 0xFFFFu;
constexpr int PL_HDR = 4;  // header words before the sites

// Words of a record in the workgroup's shared memory (a thread's slab),
// typed so that their accesses compile to LDS instructions, which wait on
// no outstanding device-memory operation (a generic access would wait for
// the previous record's stores to the pool as well).
using lds_u16 = __attribute__((address_space(3))) uint16_t;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
using lds_u4 = __attribute__((address_space(3))) u32x4;

// (STR: a record in the pool, its pieces ps words apart; else contiguous)
template <int ENC, typename W = uint16_t, bool STR = false>
struct PList {
  W *r;
  int cap;
  uint32_t ps;
  static constexpr uint32_t SM = ENC == QUTRIT ? 0x7FFFu : 0xFFFFu;
  __device__ __forceinline__ W &at(int w) const { return STR ? r[(size_t)(w >> 3) * ps + (w & 7)] : r[w]; }
  __device__ __forceinline__ int cnt() const { return at(0); }
  __device__ __forceinline__ uint32_t raw(int j) const { return at(PL_HDR + j); }
  __device__ __forceinline__ int find(uint32_t q) const {
    const int c = at(0);
    for (int j = 0; j < c; ++j)
      if ((at(PL_HDR + j) & SM) == q) return j;
    return -1;
  }
  __device__ __forceinline__ void remove(int j) {
    const int c = at(0) - 1;
    at(PL_HDR + j) = at(PL_HDR + c);
    at(0) = (uint16_t)c;
  }
  __device__ __forceinline__ void add(uint32_t x, uint32_t *err) {
    const int c = at(0);
    if (c >= cap) {
      atomicOr(err, ERR_LIST);
      return;
    }
    at(PL_HDR + c) = (uint16_t)x;
    at(0) = (uint16_t)(c + 1);
  }
  __device__ __forceinline__ void toggle(uint32_t q, uint32_t *err) {
    const int j = find(q);
    if (j >= 0)
      remove(j);
    else
      add(q, err);
  }
  // router of node v: qubit 0/1 (route left / right); qutrit -1 (W), 0 (L), 1 (R)
  __device__ __forceinline__ int dir(uint32_t v) const {
    const int j = find(2 * v);
    if (ENC == QUBIT) return j >= 0 ? 1 : 0;
    if (j < 0) return -1;
    return (at(PL_HDR + j) & LV_R_BIT) ? 1 : 0;
  }
};

// Nodes of layer l whose parent routes into them (the root for l = 0),
// collected before a qutrit store changes the list.
template <int ENC, typename W, bool STR>
__device__ __forceinline__ int gated_nodes(const PList<ENC, W, STR> &L, int l, uint32_t *gv, uint32_t *err) {
  if (l == 0) {
    gv[0] = 0;
    return 1;
  }
  int ng = 0;
  for (int j = 0; j < L.cnt(); ++j) {
    const uint32_t x = L.raw(j), q = x & PList<ENC>::SM;
    if (q & 1u) continue;
    const uint32_t p = q >> 1;
    if (layer_of(p) != l - 1) continue;
    if (ng < PL_GATED)
      gv[ng++] = 2 * p + 1 + ((x & LV_R_BIT) ? 1u : 0u);
    else
      atomicOr(err, ERR_LIST);
  }
  return ng;
}

// The gates of slice s on one component (address a).  Returns true when the
// qubit fetch flips its sign.  Every gate is a permutation of basis labels;
// it is applied entry by entry from the list as it was before the gate.
template <int ENC, typename W, bool STR>
__device__ __forceinline__ bool plain_gates(const Tables *__restrict__ tb, int s, PList<ENC, W, STR> L, uint32_t a,
                                            uint32_t *err) {
  const int n = tb->n;
  bool flip = false;
  const int ct = tb->copy_t[s];
  if (ct >= 0 && ((a >> (n - 1 - ct)) & 1u)) L.toggle(1, err);  // CNOT into d_0
  const int sl = tb->store_l[s];
  if (sl >= 0) {
    if (ENC == QUBIT) {  // SWAP(a_v, d_v) on every node of the layer
      for (int j = 0; j < L.cnt(); ++j) {
        const uint32_t q = L.raw(j);
        if (layer_of(q >> 1) == sl) L.at(PL_HDR + j) = (uint16_t)(q ^ 1u);
      }
    } else {  // (W,b) <-> (L or R by b, 0) on the gated nodes
      uint32_t gv[PL_GATED];
      const int ng = gated_nodes(L, sl, gv, err);
      for (int g = 0; g < ng && g < PL_GATED; ++g) {
        const uint32_t v = gv[g];
        const int jr = L.find(2 * v), jd = L.find(2 * v + 1);
        if (jr < 0) {  // W: the data bit moves into the router
          if (jd >= 0) {
            L.remove(jd);
            L.add(2 * v | LV_R_BIT, err);
          } else {
            L.add(2 * v, err);
          }
        } else if (jd < 0) {  // (L,0) -> (W,0), (R,0) -> (W,1)
          const bool isR = (L.raw(jr) & LV_R_BIT) != 0;
          L.remove(jr);
          if (isR) L.add(2 * v + 1, err);
        }
      }
    }
  }
  const uint32_t cm = tb->cswap[s];
  if (cm) {  // SWAP(d_v, d_child) on the layers of the slice, child by v's router
    // every router lookup below is of a node on a swap layer, so those
    // routers are collected first (up to eight; node id | R level << 15, two
    // to a register) and each data site tests them instead of scanning the
    // list (lists that collect depolarizing strays grow long); with more
    // than eight the list is scanned as usual
    int nr = 0;
    uint32_t rr0 = 0xFFFFFFFFu, rr1 = 0xFFFFFFFFu, rr2 = 0xFFFFFFFFu, rr3 = 0xFFFFFFFFu;
    for (int j = 0; j < L.cnt() && nr <= 8; ++j) {
      const uint32_t x = L.raw(j), q = x & PList<ENC>::SM;
      if (q & 1u) continue;
      const uint32_t u = q >> 1;
      if (!((cm >> layer_of(u)) & 1u)) continue;
      if (nr < 8) {
        const uint32_t tag = u | ((ENC == QUTRIT && (x & LV_R_BIT)) ? 0x8000u : 0u);
        const uint32_t sh = (uint32_t)(nr & 1) * 16u, keep = ~(0xFFFFu << sh), t = tag << sh;
        const int w = nr >> 1;
        rr0 = w == 0 ? ((rr0 & keep) | t) : rr0;
        rr1 = w == 1 ? ((rr1 & keep) | t) : rr1;
        rr2 = w == 2 ? ((rr2 & keep) | t) : rr2;
        rr3 = w == 3 ? ((rr3 & keep) | t) : rr3;
      }
      ++nr;
    }
    const bool few = nr <= 8;
    // the route of node u: qubit 0/1; qutrit -1 (W), 0 (L), 1 (R), as dir()
    auto routed = [&](uint32_t u) -> int {
      if (!few) return L.dir(u);
      bool hit = false, right = false;
      const uint32_t h[8] = {rr0 & 0xFFFFu, rr0 >> 16, rr1 & 0xFFFFu, rr1 >> 16,
                             rr2 & 0xFFFFu, rr2 >> 16, rr3 & 0xFFFFu, rr3 >> 16};
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const bool m = (h[i] & 0x7FFFu) == u;
        hit |= m;
        right |= m && (h[i] & 0x8000u);
      }
      if (ENC == QUBIT) return hit ? 1 : 0;
      return hit ? (right ? 1 : 0) : -1;
    };
    for (int j = 0; j < L.cnt(); ++j) {
      const uint32_t q = L.raw(j) & PList<ENC>::SM;
      if (!(q & 1u)) continue;
      const uint32_t v = q >> 1;
      const int l = layer_of(v);
      if ((cm >> l) & 1u) {
        const int d = routed(v);
        if (d >= 0) L.at(PL_HDR + j) = (uint16_t)(2 * (2 * v + 1 + (uint32_t)d) + 1);
      } else if (l >= 1 && ((cm >> (l - 1)) & 1u)) {
        const uint32_t p = (v - 1) >> 1;
        const int d = routed(p);
        if (d >= 0 && v == 2 * p + 1 + (uint32_t)d) L.at(PL_HDR + j) = (uint16_t)(2 * p + 1);
      }
    }
  }
  const int bb = tb->bus_b[s];
  if (bb >= 0) {  // SWAP(bus_b, d_0)
    const int j = L.find(1);
    const uint32_t bus = L.at(1);
    const bool bbit = (bus >> bb) & 1u;
    if (j >= 0 && !bbit) {
      L.remove(j);
      L.at(1) = (uint16_t)(bus | (1u << bb));
    } else if (j < 0 && bbit) {
      L.add(1, err);
      L.at(1) = (uint16_t)(bus & ~(1u << bb));
    }
  }
  const int fb = tb->fetch_b[s];
  if (fb >= 0) {
    const uint32_t v0 = (1u << (n - 1)) - 1u;
    if (ENC == QUBIT) {  // phase kickback: -1 on d_v = 1 when the routed cell holds 1
      for (int j = 0; j < L.cnt(); ++j) {
        const uint32_t q = L.raw(j);
        if (!(q & 1u) || (q >> 1) < v0) continue;
        const uint32_t v = q >> 1;
        const uint32_t cell = 2 * (v - v0) + (uint32_t)L.dir(v);
        if ((tb->mem[cell] >> fb) & 1u) flip = !flip;
      }
    } else {  // d_v ^= bit of the routed cell when r_v != W
      uint32_t gv[PL_GATED];
      int ng = 0;
      for (int j = 0; j < L.cnt(); ++j) {
        const uint32_t x = L.raw(j), q = x & PList<ENC>::SM;
        if ((q & 1u) || (q >> 1) < v0) continue;
        const uint32_t v = q >> 1;
        const uint32_t cell = 2 * (v - v0) + ((x & LV_R_BIT) ? 1u : 0u);
        if (!((tb->mem[cell] >> fb) & 1u)) continue;
        if (ng < PL_GATED)
          gv[ng++] = 2 * v + 1;
        else
          atomicOr(err, ERR_LIST);
      }
      for (int g = 0; g < ng && g < PL_GATED; ++g) L.toggle(gv[g], err);
    }
  }
  return flip;
}

// A depolarizing fault Z^b X^a on site q of one component (Sec. II B): the
// site's level x becomes x + a (mod d), then the amplitude takes
// w_d^(b (x + a)), w_2 = -1, w_3 = exp(2 pi i / 3), counted in the phase
// index ph (bit 0: a factor -1; ph >> 1: the power of w_3).  A qutrit
// router has three levels (W absent from the list, L, R with the level
// bit); every other site two.
__device__ __forceinline__ uint32_t phase_w3(uint32_t ph, uint32_t t) {
  return (ph & 1u) | ((((ph >> 1) + t) % 3u) << 1);
}

template <int ENC, typename W, bool STR>
__device__ __forceinline__ void plain_fault(PList<ENC, W, STR> L, uint32_t &ph, uint32_t q, uint32_t a, uint32_t b,
                                            uint32_t *err) {
  const bool tri = ENC == QUTRIT && (q & 1u) == 0;
  const int j = L.find(q);
  uint32_t x;
  if (!tri) {
    x = (j >= 0 ? 1u : 0u) ^ (a & 1u);
    if (a & 1u) {
      if (j >= 0)
        L.remove(j);
      else
        L.add(q, err);
    }
    if ((b & 1u) && x) ph ^= 1u;
    return;
  }
  const uint32_t v = j < 0 ? 0u : ((L.raw(j) & LV_R_BIT) ? 2u : 1u);
  x = (v + a) % 3u;
  if (v != x) {
    if (j >= 0) L.remove(j);
    if (x) L.add(q | (x == 2 ? LV_R_BIT : 0u), err);
  }
  ph = phase_w3(ph, (b * x) % 3u);
}

// (-1)^(ph & 1) w3^(ph >> 1) times z; w3 = exp(2 pi i / 3) = -1/2 + i sqrt(3)/2
__device__ __forceinline__ double2 apply_phase(double2 z, uint32_t ph) {
  if (ph & 1u) z = make_double2(-z.x, -z.y);
  const uint32_t t = ph >> 1;
  if (t) {
    const double c = -0.5, sn = t == 1 ? 0.86602540378443864676 : -0.86602540378443864676;
    z = make_double2(z.x * c - z.y * sn, z.x * sn + z.y * c);
  }
  return z;
}

// One component's slice: the gates, the slice's faults, the slice's
// damping factor a^|X| counted in the record (the count multiplied into the
// amplitude first when it would leave the power tables), and with
// candidates the hit test (returned).
template <int ENC, typename W, bool STR>
__device__ __forceinline__ int plain_slice(const Tables *__restrict__ tb, int s, PList<ENC, W, STR> L, uint32_t a,
                                           const uint32_t *__restrict__ dep, uint32_t d0, uint32_t d1,
                                           uint32_t nc, const uint32_t *cbm, double2 *ampy,
                                           const double *__restrict__ apow, int emat, uint32_t *err) {
  uint32_t ph = L.at(3);
  if (plain_gates<ENC>(tb, s, L, a, err)) ph ^= 1u;
  for (uint32_t f = d0; f < d1; ++f) {  // faults after the gates, before the damping layer
    const uint32_t e = dep[f], t = e >> 24;
    plain_fault<ENC>(L, ph, e & 0xFFFFu, t & 3u, t >> 2, err);
  }
  int e = L.at(2);
  const int cx = L.cnt();
  if (e + cx > emat) {
    const double f = apow[e];
    *ampy = make_double2(ampy->x * f, ampy->y * f);
    e = 0;
  }
  L.at(2) = (uint16_t)(e + cx);
  L.at(3) = (uint16_t)ph;
  int hit = 0;
  if (nc > 0)
    for (int j = 0; j < L.cnt() && !hit; ++j) {
      const uint32_t q = L.raw(j) & PList<ENC>::SM;
      hit = (int)((cbm[q >> 5] >> (q & 31)) & 1u);
    }
  return hit;
}

// The same on a record in device memory (one that does not fit its slab, or
// a launch without slabs): a call of its own, so that its registers do not
// add to the staged path's.
template <int ENC>
__device__ __attribute__((noinline)) int plain_slice_mem(const Tables *__restrict__ tb, int s, uint16_t *g, int lcap,
                                                         uint32_t ps, uint32_t a, const uint32_t *__restrict__ dep,
                                                         uint32_t d0, uint32_t d1, uint32_t nc, const uint32_t *cbm,
                                                         double2 *ampy, const double *__restrict__ apow, int emat,
                                                         uint32_t *err) {
  return plain_slice(tb, s, PList<ENC, uint16_t, true>{g, lcap, ps}, a, dep, d0, d1, nc, cbm, ampy, apow, emat, err);
}

struct PlainSm {
  uint32_t *cbm;     // candidate bitmap of the slice [(M + 31) / 32]
  uint32_t *cstart;  // [MAXT + 1] first candidate of each slice
  uint32_t *J;       // [JMAX] joint outcome: site | level << 16
  double *red;       // [16 * 16] reduction buffer
  int *misc;         // [16]
  int *wv;           // [4 * 16] the pick's per-wave data (up to 16 waves)
  uint16_t *slab;    // [threads * prec] one record per thread (16-byte aligned)
};

__host__ __device__ inline uint32_t plain_sm_head(int M) {
  return (uint32_t)((((M + 31) / 32) * 4 + (MAXT + 1) * 4 + JMAX * 4 + 16 * 16 * 8 + 16 * 4 + 4 * 16 * 4 + 64 + 15) & ~15);
}

__device__ inline PlainSm plain_carve(unsigned char *base, int M) {
  PlainSm s;
  size_t o = 0;
  s.red = reinterpret_cast<double *>(base + o);
  o += 16 * 16 * 8;
  s.cbm = reinterpret_cast<uint32_t *>(base + o);
  o += (size_t)((M + 31) / 32) * 4;
  s.cstart = reinterpret_cast<uint32_t *>(base + o);
  o += (MAXT + 1) * 4;
  s.J = reinterpret_cast<uint32_t *>(base + o);
  o += JMAX * 4;
  s.misc = reinterpret_cast<int *>(base + o);
  o += 16 * 4;
  s.wv = reinterpret_cast<int *>(base + o);
  s.slab = reinterpret_cast<uint16_t *>(base + plain_sm_head(M));
  return s;
}

// A record copied from the pool (its pieces ps words apart) into a thread's
// slab (sw words, a multiple of 8) in 16-byte pieces: the header words and
// the sites in use.  The
// first two pieces (the header and up to 12 sites) are loaded together,
// before the count is known.  A record
// is staged only when it fits the slab with `margin` words to spare (the
// most a slice's gates and faults can add); returns false, having copied
// only the first pieces, when it does not.
__device__ __forceinline__ bool rec_load(lds_u16 *dst, const uint16_t *__restrict__ src, uint32_t ps, int sw,
                                         int margin) {
  const u32x4 *s4 = reinterpret_cast<const u32x4 *>(src);
  const size_t pv = ps >> 3;  // (pieces apart, in 16-byte units)
  lds_u4 *d4 = (lds_u4 *)dst;
  const int nv_all = sw >> 3;
  const u32x4 v0 = s4[0];
  const u32x4 v1 = nv_all > 1 ? s4[pv] : v0;
  d4[0] = v0;
  if (nv_all > 1) d4[1] = v1;
  const uint32_t c = v0.x & 0xFFFFu;
  if (c == PL_DEAD) return true;
  if ((int)(PL_HDR + c) + margin > sw) return false;
  const int nv = (int)(PL_HDR + c + 7) >> 3;
  for (int i = 2; i < nv; i += 4) {  // longer lists: four pieces in flight at a time
    const u32x4 w0 = s4[i * pv];
    const u32x4 w1 = i + 1 < nv ? s4[(i + 1) * pv] : w0;
    const u32x4 w2 = i + 2 < nv ? s4[(i + 2) * pv] : w0;
    const u32x4 w3 = i + 3 < nv ? s4[(i + 3) * pv] : w0;
    d4[i] = w0;
    if (i + 1 < nv) d4[i + 1] = w1;
    if (i + 2 < nv) d4[i + 2] = w2;
    if (i + 3 < nv) d4[i + 3] = w3;
  }
  return true;
}

__device__ __forceinline__ void rec_store(uint16_t *__restrict__ dst, uint32_t ps, const lds_u16 *src, int sw) {
  const lds_u4 *s4 = (const lds_u4 *)src;
  u32x4 *d4 = reinterpret_cast<u32x4 *>(dst);
  const size_t pv = ps >> 3;
  const uint32_t c = src[0];
  const int nv = c == PL_DEAD ? 1 : min(sw >> 3, (int)(PL_HDR + c + 7) >> 3);
  for (int i = 0; i < nv; ++i) d4[i * pv] = s4[i];
}

__device__ __forceinline__ double abs2(double2 z) { return z.x * z.x + z.y * z.y; }

__device__ __forceinline__ double2 in_amp(const Tables *__restrict__ tb, uint32_t i) {
  return tb->cin ? make_double2(tb->cin[2 * i], tb->cin[2 * i + 1]) : make_double2(1.0 / sqrt((double)tb->D), 0.0);
}

// Exposure of branch (i, j) on its no-jump orbit through slice s, the part
// that differs between branches: its address tokens, and (qutrit) its data
// slots, which hold j_b before the fetch of bit b and j_b xor d_b after it
// (the qubit's bus words, and every router level, are common to all
// branches).
template <int ENC>
__device__ __forceinline__ int branch_exposure(const Tables *__restrict__ tb, uint32_t i, uint32_t j, int s) {
  const int n = tb->n;
  int e = 0;
  for (int t = 0; t < n; ++t)
    if ((i >> (n - 1 - t)) & 1u) e += tb->cntA[s][t];
  if (ENC == QUTRIT) {
    const uint32_t d = tb->mem[i];
    for (int b = 0; b < tb->k; ++b) {
      const int in_tree = max(0, min(s, 4 * n + 2 * b) - (2 * n + 2 * b));
      const int after = tb->cntD[s][b];
      e += (int)((j >> b) & 1u) * (in_tree - after) + (int)(((j ^ d) >> b) & 1u) * after;
    }
  }
  return e;
}

__device__ __forceinline__ uint32_t in_bus(const Tables *__restrict__ tb, uint32_t i) {
  return tb->jin ? tb->jin[i] : 0u;
}

__device__ __forceinline__ double2 camp_of(const Tables *__restrict__ tb, size_t x) {
  return make_double2(tb->camp[2 * x], tb->camp[2 * x + 1]);
}

// c_ij of the input (pair input, or the one bus word of each address)
__device__ __forceinline__ double2 in_ab(const Tables *__restrict__ tb, uint32_t i, uint32_t j) {
  if (tb->cab) {
    const size_t x = ((size_t)i << tb->k) + j;
    return make_double2(tb->cab[2 * x], tb->cab[2 * x + 1]);
  }
  return j == in_bus(tb, i) ? in_amp(tb, i) : make_double2(0.0, 0.0);
}

// WPE: the register budget, as waves per SIMD the kernel must allow (1:
// unconstrained; see plain_variant below); NT: the most threads per
// workgroup (256, or 1024 for the longest trajectories of a split run)
template <int ENC, int WPE, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE)))
k_plain(const Tables *__restrict__ tb, const Run R_) {
  const Run *rp = &R_;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int T = tb->T, M = tb->M, D = tb->D, k = tb->k;
  const int K2 = tb->K2;  // components per address (qutrit: 1, or 2^k with a pair input)
  const int kb = __ffs(K2) - 1;
  const uint32_t kmask = (1u << k) - 1u;
  const int rec = rp->prec;
  const int lcap = rec - PL_HDR;
  const bool pruned = rp->mode == 1;
  // exposures counted in a record stay within the power tables' range
  // (they are multiplied into the amplitude before they would leave it)
  const int emat = max(tb->emax, rec);
  PlainSm sm = plain_carve(smem, M);
  const uint32_t Emax = (uint32_t)(D * K2);
  uint16_t *pool = rp->pool + (size_t)blockIdx.x * Emax * rec;
  double2 *amp = reinterpret_cast<double2 *>(rp->pamp) + (size_t)blockIdx.x * Emax;
  uint8_t *hitf = rp->phit + (size_t)blockIdx.x * Emax;
  double2 *grp = reinterpret_cast<double2 *>(rp->pgrp) + ((size_t)blockIdx.x * nthr + tid) * K2;
  const double *__restrict__ apow = tb->apow + tb->emax;
  const double *__restrict__ wpow = tb->wpow + tb->emax;
  const double sg = tb->sg;
  const uint32_t ccap = rp->cand_cap;
  // the record this thread works on: staged in its slab of shared memory
  // (sw words; the gates' list scans then stay on chip) when it fits, else
  // worked on in the pool
  const int sw = (int)rp->pslab;
  uint16_t *const slab = sw ? sm.slab + (size_t)tid * sw : nullptr;
  for (int w = tid; w < (M + 31) / 32; w += nthr) sm.cbm[w] = 0u;

  // trajectories from a device queue (counter[0], cleared before the
  // launch): a workgroup that drew short ones takes more.  A split run
  // queues only the trajectories that drew a depolarizing fault (their
  // segment of the order); the trajectory kernel runs the others.
  const uint32_t q0 = rp->dsplit ? rp->bucket_base[MAXB] : 0u;
  const uint32_t qn = rp->dsplit ? rp->bucket_base[MAXB + 1] - q0 : rp->ntraj;
  for (;;) {
    if (tid == 0) sm.misc[12] = (int)atomicAdd(&rp->counter[0], 1u);
    __syncthreads();  // (misc[12] is written again only after the trajectory's last barrier)
    const uint32_t slot = (uint32_t)sm.misc[12];
    if (slot >= qn) break;
    const uint32_t tj = rp->dsplit ? rp->order[q0 + slot] : slot;
    const uint32_t traj = rp->traj0 + tj;
    const uint32_t nct = min(rp->ncand[tj], ccap);
    const uint32_t *__restrict__ cand = rp->cand + (size_t)tj * ccap;
    const uint32_t ref = rp->ref[tj];
    // explicit addresses: every address (full), or the bad ones plus the
    // reference in ascending order (pruned, Alg. 1); explicit component y =
    // g * K2 + beta of explicit address xl[g]
    const uint16_t *__restrict__ xl = pruned ? rp->xlist + (size_t)tj * D : nullptr;
    const uint32_t A = pruned ? (rp->nexpl[tj] >> kb) : (uint32_t)D;
    const uint32_t E = A * (uint32_t)K2;
    const uint32_t ps = E * 8u;  // words between the pieces of a record in the pool
    const uint64_t *__restrict__ badg = rp->badbits + (size_t)tj * ((D + 63) >> 6);
    // the good branches ride on the reference (pruned, a reference exists)
    const bool goods = pruned && ref != 0xFFFFFFFFu && A < (uint32_t)D;
    if (tid == 0) sm.misc[8] = -1;
    for (uint32_t j = tid; j <= nct; j += nthr) {  // first candidate of each slice
      const int sj = j < nct ? (int)(cand[j] / (uint32_t)M) + 1 : T;
      const int sp = j > 0 ? (int)(cand[j - 1] / (uint32_t)M) + 1 : 0;
      for (int ss = sp + 1; ss <= sj; ++ss) sm.cstart[ss] = j;
    }
    __syncthreads();
    // the input after the first wall: qubit, the 2^k bus words beta of each
    // address i with amplitude c_i 2^(-k/2) (-1)^(beta . j_i); qutrit, bus
    // word j_i with amplitude c_i.  The data-loading input has c_i =
    // 2^(-n/2), j_i = 0; an address absent from the input has no component.
    // A pair input sum_ij c_ij |i>|j> comes with each component's amplitude
    // (qubit: 2^(-k/2) sum_j c_ij (-1)^(beta . j), alive with its address;
    // qutrit: c_ij, alive when nonzero).
    const double wall = ENC == QUBIT ? 1.0 / sqrt((double)K2) : 1.0;
    for (uint32_t y = tid; y < E; y += nthr) {
      uint16_t *r = pool + (size_t)y * 8;  // (the header: piece 0)
      const uint32_t g = y >> kb, beta = y & (uint32_t)(K2 - 1);
      const uint32_t i = xl ? xl[g] : g;
      if (i == ref) sm.misc[8] = (int)g;
      if (tb->camp) {
        const double2 c = camp_of(tb, ((size_t)i << kb) + beta);
        const bool alive = ENC == QUBIT ? (tb->aflag[i] & 1u) != 0 : (c.x != 0.0 || c.y != 0.0);
        r[0] = alive ? 0 : PL_DEAD;
        r[1] = (uint16_t)beta;
        r[2] = 0;
        r[3] = 0;
        amp[y] = c;
        continue;
      }
      double2 c = in_amp(tb, i);
      const uint32_t j = in_bus(tb, i);
      if (ENC == QUBIT && (__popc(beta & j) & 1)) c = make_double2(-c.x, -c.y);
      r[0] = (c.x != 0.0 || c.y != 0.0) ? 0 : PL_DEAD;
      r[1] = (uint16_t)(ENC == QUBIT ? beta : j);
      r[2] = 0;
      r[3] = 0;
      amp[y] = make_double2(c.x * wall, c.y * wall);
    }
    const uint32_t nd = rp->dep ? min(rp->ndep[tj], rp->dep_cap) : 0u;
    const uint32_t *__restrict__ dep = rp->dep ? rp->dep + (size_t)tj * rp->dep_cap : nullptr;
    uint32_t dpos = 0;
    int njumps = 0, first_jump = 0;
    uint32_t jl_n = 0;
    __syncthreads();
    const int gref = sm.misc[8];  // explicit index of the reference, or -1
    const uint32_t jref = goods ? in_bus(tb, ref) : 0u;
    double cref2 = 0.0;
    if (goods) cref2 = abs2(in_amp(tb, ref));
    auto is_bad = [&](uint32_t i) -> bool { return (badg[i >> 6] >> (i & 63)) & 1ull; };
    // explicit component y's weight |A|^2 before the current slice's
    // damping layer (its record counts that layer's a^|X| already), and its
    // amplitude with every counted factor multiplied in
    auto wt = [&](uint32_t y) -> double {
      const uint16_t *r = pool + (size_t)y * 8;
      return abs2(amp[y]) * wpow[(int)r[2] - (int)r[0]];
    };
    auto amp_of = [&](uint32_t y) -> double2 {
      const uint16_t *r = pool + (size_t)y * 8;
      const double f = apow[r[2]];
      return apply_phase(make_double2(amp[y].x * f, amp[y].y * f), r[3]);
    };
    // The predicted branches (good, present, not the reference) relative to
    // the reference, through slice s: the sum over branches (i, j) holding
    // one bus word of |c_ij / c_ref|^2 (1-gamma)^(e(i,j) - e(ref)) (qutrit
    // pair input: every (address, bus word) pair is such a branch).  Good
    // qubit addresses holding several bus words enter bus word by bus word
    // below (multi_sum).
    auto good_sum = [&](int s, int eref) -> double {
      double acc = 0.0;
      if (ENC == QUTRIT && tb->cab) {
        for (uint32_t x = (uint32_t)tid; x < ((uint32_t)D << kb); x += (uint32_t)nthr) {
          const uint32_t i = x >> kb, j = x & (uint32_t)(K2 - 1);
          if (i == ref || is_bad(i)) continue;
          const double c2 = abs2(in_ab(tb, i, j));
          if (c2 != 0.0) acc += c2 / cref2 * wpow[branch_exposure<ENC>(tb, i, j, s) - eref];
        }
        return acc;
      }
      for (int ii = tid; ii < D; ii += nthr) {
        const uint32_t i = (uint32_t)ii;
        if (i == ref || is_bad(i)) continue;
        const double c2 = abs2(in_amp(tb, i));  // (0 for an address holding several bus words)
        if (c2 != 0.0) acc += c2 / cref2 * wpow[branch_exposure<ENC>(tb, i, in_bus(tb, i), s) - eref];
      }
      return acc;
    };
    // qubit, good addresses holding several bus words: component (i, beta)
    // has the reference's component beta times camp(i, beta) / camp(ref,
    // beta) a^(e(i) - e(ref)) (Theorem 3); its weight through slice s
    auto multi_ratio = [&](uint32_t i, uint32_t beta, int s, int eref) -> double {
      const double f = abs2(camp_of(tb, ((size_t)i << kb) + beta)) / abs2(camp_of(tb, ((size_t)ref << kb) + beta));
      return f * wpow[branch_exposure<ENC>(tb, i, 0u, s) - eref];
    };
    // ... summed over those addresses, split by whether the reference's
    // component is hit (a good branch carries no excitation of its own on a
    // candidate site, but it shares the reference's strays: an X-type fault
    // on an idle site excites every branch off its range alike)
    auto multi_sum = [&](int s, int eref, double &we, double &wh) {
      if (ENC != QUBIT || !tb->cab) return;
      for (uint32_t z = (uint32_t)tid; z < ((uint32_t)D << kb); z += (uint32_t)nthr) {
        const uint32_t i = z >> kb, beta = z & (uint32_t)(K2 - 1);
        if (tb->aflag[i] != 1u || is_bad(i)) continue;  // present, several bus words
        const uint32_t yr = (uint32_t)gref * K2 + beta;
        if (pool[(size_t)yr * 8] == PL_DEAD) continue;
        const double w = multi_ratio(i, beta, s, eref) * wt(yr);
        if (hitf[yr])
          wh += w;
        else
          we += w;
      }
    };
    // weight of good label (a, beta) relative to the reference component it
    // follows (index yr), through slice s; 0 for a label that is no branch
    auto good_label = [&](uint32_t a, uint32_t beta, int s, int eref, uint32_t &yr) -> double {
      if (ENC == QUBIT) {
        yr = (uint32_t)gref * K2 + beta;
        if (tb->aflag && tb->aflag[a] == 1u) return multi_ratio(a, beta, s, eref);
        const double c2 = abs2(in_amp(tb, a));
        return c2 == 0.0 ? 0.0 : c2 / cref2 * wpow[branch_exposure<ENC>(tb, a, 0u, s) - eref];
      }
      yr = (uint32_t)gref * K2 + (tb->cab ? jref : 0u);
      const double c2 = tb->cab ? abs2(in_ab(tb, a, beta)) : abs2(in_amp(tb, a));
      const uint32_t j = tb->cab ? beta : in_bus(tb, a);
      return c2 == 0.0 ? 0.0 : c2 / cref2 * wpow[branch_exposure<ENC>(tb, a, j, s) - eref];
    };

    for (int s = 1; s < T; ++s) {
      const uint32_t cb = sm.cstart[s], ce = sm.cstart[s + 1];
      const uint32_t nc = ce - cb;
      const uint32_t d0 = dpos;  // the slice's depolarizing faults: dep[d0 .. dpos)
      while (dpos < nd && ((dep[dpos] >> 16) & 0xFFu) == (uint32_t)s) ++dpos;
      for (uint32_t j = cb + tid; j < ce; j += nthr) {
        const uint32_t q = cand[j] - (uint32_t)(s - 1) * M;
        atomicOr(&sm.cbm[q >> 5], 1u << (q & 31));
      }
      __syncthreads();
      // gates and faults, then (without candidates) K0 at once; with
      // candidates the hit test of every component against the slice's set
      int anyhit = 0;
      // a slice adds at most: qubit, the copy and bus-swap sites; qutrit,
      // those and one per gated node of a store and of a fetch; one per fault
      const int margin = (ENC == QUTRIT ? 2 + 2 * PL_GATED : 2) + (int)(dpos - d0);
      // (the slice's K_0 = a^|X| joins each record's exposure; a jump takes
      // back its sites' share below)
      for (uint32_t y = tid; y < E; y += nthr) {
        uint16_t *const g = pool + (size_t)y * 8;
        const uint32_t a = xl ? xl[y >> kb] : (y >> kb);
        int hit;
        if (slab && rec_load((lds_u16 *)slab, g, ps, sw, margin)) {
          PList<ENC, lds_u16> L{(lds_u16 *)slab, sw - PL_HDR};
          if (L.cnt() == PL_DEAD) continue;
          hit = plain_slice(tb, s, L, a, dep, d0, dpos, nc, sm.cbm, amp + y, apow, emat, rp->err);
          rec_store(g, ps, (lds_u16 *)slab, sw);
        } else {
          if (g[0] == PL_DEAD) continue;
          hit = plain_slice_mem<ENC>(tb, s, g, lcap, ps, a, dep, d0, dpos, nc, sm.cbm, amp + y, apow, emat,
                                     rp->err);
        }
        if (nc > 0) {
          hitf[y] = (uint8_t)hit;
          anyhit |= hit;
        }
      }
      if (nc == 0) continue;  // (the bitmap is already clean)
      anyhit = __syncthreads_or(anyhit);
      int nJ = 0;
      if (anyhit) {
        // Eq. maskweight: the empty-mask block and the hit components; a
        // good branch has the reference's mask for the same bus word and the
        // reference's weight times its ratio
        // empty, hit, ref empty, ref hit, ratio sum, predicted several-word
        // weight not hit and hit
        double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (uint32_t y = tid; y < E; y += nthr) {
          if (pool[(size_t)y * 8] == PL_DEAD) continue;
          const double w = wt(y);
          const int h = hitf[y] ? 1 : 0;
          acc[h] += w;
          if (goods && (int)(y >> kb) == gref) acc[2 + h] += w;
        }
        // the weights before this slice's damping layer: exposures through s-1
        const int eref = goods ? branch_exposure<ENC>(tb, ref, jref, s - 1) : 0;
        if (goods) {
          acc[4] = good_sum(s - 1, eref);
          multi_sum(s - 1, eref, acc[5], acc[6]);
        }
        block_sum<7>(acc, sm.red);
        // a good branch is hit exactly when the reference's component it
        // follows is
        const double w_empty = acc[0] + acc[4] * acc[2] + acc[5];
        const double w_hit = acc[1] + acc[4] * acc[3] + acc[6];
        const double u = rp->forced ? rp->uaux[s] : uniform53(rp->seed, (uint32_t)s, 0, traj, 2u);
        const double r = u * (w_empty + w_hit);
        if (!(r < w_empty)) {
          // x*: first hit component, in initial-label order over every
          // branch, whose running weight exceeds r - w(empty); the last hit
          // one if rounding runs out.  pick = (label, explicit index whose
          // list holds x*'s mask)
          const double r2 = r - w_empty;
          double base = 0.0;
          int pick = -1, last = -1, pick_y = -1, last_y = -1;
          // Only a hit reference component makes good labels candidates for
          // x*; otherwise the explicit components alone, which are in label
          // order already (ascending explicit addresses), are scanned.
          const bool labels = goods && (acc[3] > 0.0 || acc[6] > 0.0);
          const uint32_t Lx = labels ? (uint32_t)(D * K2) : E;
          for (uint32_t x0 = 0; x0 < Lx && pick < 0; x0 += (uint32_t)nthr) {
            const uint32_t x = x0 + (uint32_t)tid;
            double w = 0.0;
            int my = -1;
            if (x < Lx && !labels) {
              if (pool[(size_t)x * 8] != PL_DEAD && hitf[x]) {
                w = wt(x);
                my = (int)x;
              }
            } else if (x < Lx) {
              const uint32_t a = x >> kb, beta = x & (uint32_t)(K2 - 1);
              int g = -1;
              if (!xl || A == (uint32_t)D) {  // (every address explicit, in order)
                g = (int)a;
              } else if (a == ref || is_bad(a)) {
                int lo = 0, hi = (int)A - 1;  // a's position in the ascending explicit list
                while (lo < hi) {
                  const int mid = (lo + hi) >> 1;
                  if (xl[mid] < a)
                    lo = mid + 1;
                  else
                    hi = mid;
                }
                g = lo;
              }
              if (g >= 0) {
                const uint32_t y = (uint32_t)g * K2 + beta;
                if (pool[(size_t)y * 8] != PL_DEAD && hitf[y]) {
                  w = wt(y);
                  my = (int)y;
                }
              } else if (goods) {  // a good label follows the reference's component
                uint32_t yr = 0;
                const double rw = good_label(a, beta, s - 1, eref, yr);
                if (rw > 0.0 && pool[(size_t)yr * 8] != PL_DEAD && hitf[yr]) {
                  w = wt(yr) * rw;
                  if (w > 0.0) my = (int)yr;
                }
              }
            }
            __syncthreads();  // (the scan buffer is reused)
            const double ex = block_excl_scan(w, sm.red);
            __syncthreads();
            if (tid == nthr - 1) sm.red[64] = ex + w;
            const bool mine = my >= 0 && base + ex + w > r2;
            int lowest = mine ? (int)x : 0x7FFFFFFF;
            for (int off = 32; off > 0; off >>= 1) lowest = min(lowest, __shfl_xor(lowest, off, 64));
            int lastm = my >= 0 ? (int)x : -1;
            for (int off = 32; off > 0; off >>= 1) lastm = max(lastm, __shfl_xor(lastm, off, 64));
            if ((tid & 63) == 0) {
              sm.wv[tid >> 6] = lowest;
              sm.wv[32 + (tid >> 6)] = lastm;
            }
            if (mine && (int)x == lowest) sm.wv[16 + (tid >> 6)] = my;  // explicit index of the wave's pick
            if (my >= 0 && (int)x == lastm) sm.wv[48 + (tid >> 6)] = my;
            __syncthreads();
            int best = 0x7FFFFFFF, bw = -1, lw = -1, lst = -1;
            for (int w8 = 0; w8 < nthr / 64; ++w8) {
              if (sm.wv[w8] < best) {
                best = sm.wv[w8];
                bw = w8;
              }
              const int l8 = sm.wv[32 + w8];
              if (l8 > lst) {
                lst = l8;
                lw = w8;
              }
            }
            if (lst >= 0 && lst > last) {
              last = lst;
              last_y = sm.wv[48 + lw];
            }
            base += sm.red[64];
            if (best != 0x7FFFFFFF) {
              pick = best;
              pick_y = sm.wv[16 + bw];
            }
            __syncthreads();
          }
          if (pick < 0) pick_y = last_y;
          // J = the slice's candidates among x*'s excited sites, with levels
          if (tid == 0) {
            PList<ENC, uint16_t, true> L{pool + (size_t)pick_y * 8, lcap, ps};
            int m = 0;
            for (int j = 0; j < L.cnt(); ++j) {
              const uint32_t x = L.raw(j), q = x & PList<ENC>::SM;
              if (!((sm.cbm[q >> 5] >> (q & 31)) & 1u)) continue;
              const uint32_t lev = (ENC == QUTRIT && (x & LV_R_BIT)) ? 2u : 1u;
              if (m < JMAX) sm.J[m++] = q | (lev << 16);
            }
            for (int i = 1; i < m; ++i)  // ascending site order
              for (int j = i; j > 0 && (sm.J[j] & 0xFFFFu) < (sm.J[j - 1] & 0xFFFFu); --j) {
                const uint32_t t = sm.J[j];
                sm.J[j] = sm.J[j - 1];
                sm.J[j - 1] = t;
              }
            sm.misc[0] = m;
          }
          __syncthreads();
          nJ = sm.misc[0];
        }
      }
      // K_J on every explicit component after a jump: survivors carry J's
      // sites at J's levels (the good branches survive exactly when the
      // reference does) and take sqrt(gamma)^|J| a^(|X| - |J|), the record
      // having counted a^|X| for the slice.  Without a jump K_0 = a^|X| is
      // counted already.
      for (uint32_t y = tid; nJ > 0 && y < E; y += nthr) {
        uint16_t *const g = pool + (size_t)y * 8;
        if (g[0] == PL_DEAD) continue;
        // (a jump changes few entries: the record is edited in place)
        PList<ENC, uint16_t, true> L{g, lcap, ps};
        bool ok = true;
        for (int c = 0; c < nJ && ok; ++c) {
          const uint32_t q = sm.J[c] & 0xFFFFu, lev = sm.J[c] >> 16;
          const int j = L.find(q);
          ok = j >= 0 && ((ENC == QUTRIT && (L.raw(j) & LV_R_BIT)) ? 2u : 1u) == lev;
        }
        if (!ok) {
          g[0] = PL_DEAD;
          amp[y] = make_double2(0.0, 0.0);
          continue;
        }
        double f = 1.0;
        for (int c = 0; c < nJ; ++c) f *= sg;
        amp[y] = make_double2(amp[y].x * f, amp[y].y * f);
        for (int c = 0; c < nJ; ++c) L.remove(L.find(sm.J[c] & 0xFFFFu));
        g[2] = (uint16_t)(g[2] - nJ);
      }
      if (nJ > 0) {
        ++njumps;
        if (!first_jump) first_jump = s;
        if (rp->jlog && tid == 0)
          for (int c = 0; c < nJ; ++c, ++jl_n)
            if (jl_n < rp->jcap) rp->jlog[(size_t)tj * rp->jcap + jl_n] = sm.J[c] | ((uint32_t)s << 24);
      }
      __syncthreads();
      for (uint32_t j = cb + tid; j < ce; j += nthr) {  // leave the bitmap clean
        const uint32_t q = cand[j] - (uint32_t)(s - 1) * M;
        sm.cbm[q >> 5] = 0u;
      }
      __syncthreads();
    }

    // the last slice may have ended without a barrier (no candidates): every
    // thread's lists must be final before any thread reads another's
    __syncthreads();
    if (rp->exp && tj == 0) {  // test entry: every explicit component's final list and amplitude
      const uint32_t rw = 3u + (uint32_t)tb->lmax;
      for (uint32_t y = tid; y < E; y += nthr) {
        uint16_t *const r = pool + (size_t)y * 8;
        const PList<ENC, uint16_t, true> L{r, lcap, ps};
        const uint32_t a = xl ? xl[y >> kb] : (y >> kb);
        const uint32_t x = (a << kb) | (y & (uint32_t)(K2 - 1));
        uint32_t *o = rp->exp + (size_t)x * rw;
        if (r[0] == PL_DEAD) continue;
        if (r[0] > (uint32_t)tb->lmax) atomicOr(rp->err, ERR_LIST);  // (strays: more sites than an export record holds)
        const uint32_t m = min((uint32_t)r[0], (uint32_t)tb->lmax);
        o[0] = a | ((uint32_t)r[1] << 16) | EXP_PRESENT;
        o[1] = 0;
        o[2] = m;
        for (uint32_t j = 0; j < m; ++j) {
          const uint32_t e = L.raw(j);
          const uint32_t q = e & PList<ENC>::SM, lev = (ENC == QUTRIT && (e & LV_R_BIT)) ? 2u : 1u;
          o[3 + j] = q | (lev << 16);
        }
        if (rp->expamp) {
          const double2 at = amp_of(y);
          rp->expamp[2 * x] = at.x;
          rp->expamp[2 * x + 1] = at.y;
        }
      }
    }
    // second wall (qubit), tree measurement, fidelity.  Components with an
    // excited tree are orthogonal to the ideal output and to every other
    // group, so only their weight counts; the ground components of an
    // address are grouped by bus word (before the wall, qubit).  The ideal
    // output is sum_ij c_ij |i>|j xor d_i>|ground>: overlap terms
    // conj(c_{i, w xor d_i}) A(i, w) over the output words w.  The
    // reference's own terms are kept apart as well: a predicted branch
    // (i, j) adds |c_ij|^2 a^(e - e_ref) / |c_ref|^2 times the reference's
    // overlap term and |c_ij / c_ref|^2 (1-gamma)^(e - e_ref) times its
    // weights (Theorem 3 with the XOR mirror, Proposition 1).  With
    // truncation, the output words of every good address but the reference
    // that lie more than trunc_w bit flips from its ideal word are dropped
    // (Sec. V); the reference's weight within that radius carries the
    // predicted branches.
    const int tw = ENC == QUBIT ? tb->trunc_w : -1;
    double fin[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    // overlap re, im, w_ground, w_excited, ref alive, ref overlap re, im,
    // ref w_ground, ref w_excited, ratio sums (below), ref w_ground within
    // the truncation radius
    const int nw = (ENC == QUBIT || tb->cab) ? K2 : 1;  // output words held per address
    for (uint32_t g = (uint32_t)tid; g < A; g += (uint32_t)nthr) {
      const uint32_t i = xl ? xl[g] : g;
      const bool isref = i == ref;
      const uint32_t want = (in_bus(tb, i) ^ tb->mem[i]) & kmask;
      const bool trunc = tw >= 0 && !isref && !is_bad(i);
      bool any = false;
      for (int b = 0; b < nw; ++b) grp[b] = make_double2(0.0, 0.0);
      for (int b = 0; b < K2; ++b) {
        const uint32_t y = g * (uint32_t)K2 + (uint32_t)b;
        const uint16_t *r = pool + (size_t)y * 8;
        if (r[0] == PL_DEAD) continue;
        if (isref) fin[4] = 1.0;
        const double2 at = amp_of(y);
        if (r[0] != 0) {
          fin[3] += abs2(at);
          if (isref) fin[8] += abs2(at);
          continue;
        }
        // qutrit with one component per address: slot 0, holding it only
        // when its bus word is the ideal one
        if (nw == 1 && ((uint32_t)r[1] & kmask) != want) {
          fin[2] += abs2(at);
          if (isref) {
            fin[7] += abs2(at);
            fin[10] += abs2(at);
          }
          continue;
        }
        const uint32_t bw = nw == 1 ? 0u : ((uint32_t)r[1] & (uint32_t)(nw - 1));
        grp[bw] = make_double2(grp[bw].x + at.x, grp[bw].y + at.y);
        any = true;
      }
      if (!any) continue;
      if (ENC == QUBIT)
        for (int len = 1; len < K2; len <<= 1)  // Walsh-Hadamard transform in place
          for (int b = 0; b < K2; ++b)
            if (!(b & len)) {
              const double2 u = grp[b], v = grp[b + len];
              grp[b] = make_double2(u.x + v.x, u.y + v.y);
              grp[b + len] = make_double2(u.x - v.x, u.y - v.y);
            }
      const double h = ENC == QUBIT ? 1.0 / sqrt((double)K2) : 1.0;
      for (int c = 0; c < nw; ++c) {
        const double2 v = make_double2(grp[c].x * h, grp[c].y * h);
        const int dist = __popc(((uint32_t)c ^ want) & kmask);
        if (trunc && dist > tw) continue;
        fin[2] += abs2(v);
        if (isref) {
          fin[7] += abs2(v);
          if (tw < 0 || dist <= tw) fin[10] += abs2(v);
        }
        // the input amplitude whose ideal output word is c
        const double2 ci = nw == 1 ? in_amp(tb, i) : in_ab(tb, i, ((uint32_t)c ^ tb->mem[i]) & kmask);
        const double ox = ci.x * v.x + ci.y * v.y, oy = ci.x * v.y - ci.y * v.x;  // conj(ci) v
        fin[0] += ox;
        fin[1] += oy;
        if (isref) {
          fin[5] += ox;
          fin[6] += oy;
        }
      }
    }
    double gw = 0.0, ga = 0.0;  // sums over predicted branches of (1-gamma)^de |c/c_ref|^2 and a^de |c|^2
    if (goods) {
      const int eref = branch_exposure<ENC>(tb, ref, jref, T - 1);
      if (ENC == QUTRIT && tb->cab) {
        for (uint32_t x = (uint32_t)tid; x < ((uint32_t)D << kb); x += (uint32_t)nthr) {
          const uint32_t i = x >> kb, j = x & (uint32_t)(K2 - 1);
          if (i == ref || is_bad(i)) continue;
          const double c2 = abs2(in_ab(tb, i, j));
          if (c2 == 0.0) continue;
          const int de = branch_exposure<ENC>(tb, i, j, T - 1) - eref;
          gw += c2 / cref2 * wpow[de];
          ga += c2 * apow[de];
        }
      } else {
        for (int ii = tid; ii < D; ii += nthr) {
          const uint32_t i = (uint32_t)ii;
          if (i == ref || is_bad(i)) continue;
          const double c2 = abs2(in_amp(tb, i));
          if (c2 == 0.0) continue;
          const int de = branch_exposure<ENC>(tb, i, in_bus(tb, i), T - 1) - eref;
          gw += c2 / cref2 * wpow[de];
          ga += c2 * apow[de];
        }
      }
      // qubit, good addresses holding several bus words: component (i,
      // beta) = camp(i, beta) / camp(ref, beta) a^(e(i) - e(ref)) (-1)^(beta
      // . (d_i xor d_ref)) times the reference's, then the wall (O(k 2^k)
      // per address, Table 2)
      if (ENC == QUBIT && tb->cab && gref >= 0)
        for (int ii = tid; ii < D; ii += nthr) {
          const uint32_t i = (uint32_t)ii;
          if (tb->aflag[i] != 1u || is_bad(i)) continue;
          const int de = branch_exposure<ENC>(tb, i, 0u, T - 1) - eref;
          const uint32_t dd = (tb->mem[i] ^ tb->mem[ref]) & kmask;
          bool any = false;
          for (int b = 0; b < K2; ++b) {
            const uint32_t yr = (uint32_t)gref * K2 + (uint32_t)b;
            const uint16_t *r = pool + (size_t)yr * 8;
            grp[b] = make_double2(0.0, 0.0);
            if (r[0] == PL_DEAD) continue;
            const double2 ca = camp_of(tb, ((size_t)i << kb) + b), cr = camp_of(tb, ((size_t)ref << kb) + b);
            const double den = abs2(cr);
            if (r[0] != 0) {  // (an excited reference: the mirrored branch is excited too)
              fin[3] += abs2(ca) / den * wpow[de] * abs2(amp_of(yr));
              continue;
            }
            // q = ca / cr a^de (+-1), then times the reference's amplitude
            const double qx = (ca.x * cr.x + ca.y * cr.y) / den, qy = (ca.y * cr.x - ca.x * cr.y) / den;
            const double f = apow[de] * ((__popc((uint32_t)b & dd) & 1) ? -1.0 : 1.0);
            const double2 u = amp_of(yr);
            grp[b] = make_double2(f * (qx * u.x - qy * u.y), f * (qx * u.y + qy * u.x));
            any = true;
          }
          if (!any) continue;
          for (int len = 1; len < K2; len <<= 1)
            for (int b = 0; b < K2; ++b)
              if (!(b & len)) {
                const double2 u = grp[b], v = grp[b + len];
                grp[b] = make_double2(u.x + v.x, u.y + v.y);
                grp[b + len] = make_double2(u.x - v.x, u.y - v.y);
              }
          const double h = 1.0 / sqrt((double)K2);
          for (int c = 0; c < K2; ++c) {
            const double2 v = make_double2(grp[c].x * h, grp[c].y * h);
            fin[2] += abs2(v);
            const double2 ci = in_ab(tb, i, ((uint32_t)c ^ tb->mem[i]) & kmask);
            fin[0] += ci.x * v.x + ci.y * v.y;
            fin[1] += ci.x * v.y - ci.y * v.x;
          }
        }
    }
    fin[9] = gw;
    double fin2[1] = {ga};
    block_sum<11>(fin, sm.red);
    block_sum<1>(fin2, sm.red + 11 * 16);  // (after the 16 waves' entries of the first)
    if (tid == 0) {
      double ovx = fin[0], ovy = fin[1], wg = fin[2], wx = fin[3];
      if (goods && cref2 > 0.0) {
        const double ga_ref = fin2[0] / cref2;
        ovx += ga_ref * fin[5];
        ovy += ga_ref * fin[6];
        wg += fin[9] * fin[10];  // (fin[10] = fin[7] without truncation)
        wx += fin[9] * fin[8];
      }
      const double ov2 = ovx * ovx + ovy * ovy;
      const double wt = wg + wx;
      const double uf = rp->forced ? rp->ufin : uniform53(rp->seed, 0, 0, traj, 3u);
      const bool qg = uf * wt < wg;
      rp->fid[tj] = (qg && wg > 0.0) ? ov2 / wg : 0.0;
      if (rp->jn) rp->jn[tj] = jl_n;
      if (rp->st) {
        qram_traj_stats o;
        o.n_cand = rp->ncand[tj];
        o.n_bad = rp->nbad[tj];
        o.ref_addr = ref;
        o.n_explicit = E;
        o.n_jumps = (uint16_t)njumps;
        o.first_jump_slice = (uint16_t)first_jump;
        o.ref_survived = (uint8_t)(ref != 0xFFFFFFFFu && fin[4] > 0.0);
        o.q_ground = (uint8_t)qg;
        o.flags = (uint8_t)((rp->ncand[tj] > ccap ? 1 : 0));
        o.pad = 0;
        o.fid_pre = wt > 0.0 ? ov2 / wt : 0.0;
        rp->st[tj] = o;
      }
    }
    __syncthreads();
  }
}

}  // namespace

uint32_t plain_lds_bytes(int M, uint32_t slab_words) { return plain_sm_head(M) + slab_words * 2u; }

// Register budgets of the plain kernel, tried in this order: unconstrained
// (about 150 registers, three waves per SIMD), at most 128 registers (four
// waves) and, qubit only, at most 96 (five).  The capped builds spill a few
// words outside the record loop; they pay where registers, not shared
// memory, limit the workgroups a compute unit holds (short records in
// small slabs).  A launch takes the first budget that fits the workgroups
// per compute unit it asks for, else the one that fits the most.
// Workgroups of more than 256 threads (up to 1024) take a build of their
// own, at most 128 registers.
namespace {
template <int ENC, int WPE, int NT>
int plain_occ_one(int threads, uint32_t lds_bytes) {
  int blocks = 0;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_plain<ENC, WPE, NT>, threads, lds_bytes) ==
                 hipSuccess
             ? blocks
             : 0;
}
constexpr int PLAIN_BIG = 3;  // the variant of the large workgroups
int plain_occ_variant(int enc, int threads, uint32_t lds_bytes, int v) {
  if (v == PLAIN_BIG)
    return enc == QUBIT ? plain_occ_one<QUBIT, 4, 1024>(threads, lds_bytes)
                        : plain_occ_one<QUTRIT, 4, 1024>(threads, lds_bytes);
  if (enc == QUBIT)
    return v == 0 ? plain_occ_one<QUBIT, 1, 256>(threads, lds_bytes)
                  : (v == 1 ? plain_occ_one<QUBIT, 4, 256>(threads, lds_bytes)
                            : plain_occ_one<QUBIT, 5, 256>(threads, lds_bytes));
  return v == 0 ? plain_occ_one<QUTRIT, 1, 256>(threads, lds_bytes) : plain_occ_one<QUTRIT, 4, 256>(threads, lds_bytes);
}
}  // namespace

hipError_t plain_prepare(int lds_max) {
  hipError_t e = hipSuccess;
  const void *fns[2] = {reinterpret_cast<const void *>(&k_plain<QUBIT, 4, 1024>),
                        reinterpret_cast<const void *>(&k_plain<QUTRIT, 4, 1024>)};
  for (const void *f : fns) {  // the large workgroups' slabs may pass 64 KiB
    hipFuncAttributes fa;
    int dyn = lds_max;
    if (hipFuncGetAttributes(&fa, f) == hipSuccess) dyn = lds_max - (int)fa.sharedSizeBytes;
    const hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    if (r != hipSuccess) e = r;
  }
  return e;
}

int plain_variant(int enc, int threads, uint32_t lds_bytes, int per_cu, int &occ) {
  if (threads > 256) {
    occ = plain_occ_variant(enc, threads, lds_bytes, PLAIN_BIG);
    return PLAIN_BIG;
  }
  int var = 0;
  occ = 0;
  for (int v = 0; v < (enc == QUBIT ? 3 : 2); ++v) {
    const int o = plain_occ_variant(enc, threads, lds_bytes, v);
    if (o >= per_cu) {
      occ = o;
      return v;
    }
    if (o > occ) {
      occ = o;
      var = v;
    }
  }
  return var;
}

int plain_occupancy(int enc, int threads, uint32_t lds_bytes) {
  int occ = 0;
  plain_variant(enc, threads, lds_bytes, 1 << 30, occ);
  return occ;
}

hipError_t launch_plain(const Tables *tb, const Run &rp, int enc, int variant, uint32_t grid, int threads,
                        uint32_t lds_bytes, hipStream_t s) {
  const hipError_t e = launch_fill_u32(rp.counter, 0u, 1u, s);  // the queue head
  if (e != hipSuccess) return e;
  const dim3 g(grid), b(threads);
  if (enc == QUBIT) {
    if (variant == PLAIN_BIG)
      hipLaunchKernelGGL((k_plain<QUBIT, 4, 1024>), g, b, lds_bytes, s, tb, rp);
    else if (variant == 2)
      hipLaunchKernelGGL((k_plain<QUBIT, 5, 256>), g, b, lds_bytes, s, tb, rp);
    else if (variant == 1)
      hipLaunchKernelGGL((k_plain<QUBIT, 4, 256>), g, b, lds_bytes, s, tb, rp);
    else
      hipLaunchKernelGGL((k_plain<QUBIT, 1, 256>), g, b, lds_bytes, s, tb, rp);
  } else {
    if (variant == PLAIN_BIG)
      hipLaunchKernelGGL((k_plain<QUTRIT, 4, 1024>), g, b, lds_bytes, s, tb, rp);
    else if (variant == 1)
      hipLaunchKernelGGL((k_plain<QUTRIT, 4, 256>), g, b, lds_bytes, s, tb, rp);
    else
      hipLaunchKernelGGL((k_plain<QUTRIT, 1, 256>), g, b, lds_bytes, s, tb, rp);
  }
  return hipGetLastError();
}

}  // namespace qr
