// Trajectory evolution kernel (gfx950): one workgroup per trajectory carries
// every explicit component through the T-1 slices of the schedule with one
// joint damping layer per slice (Eq. layerkraus, Theorem 4, Eq. maskweight),
// predicts the good branches in pruned mode (Proposition 1, Theorem 3), and
// reduces the post-measurement fidelity (Alg. 1 steps 3-6).
//
// Components never split between the walls: every gate permutes basis labels
// and K_J maps survivors one to one.  A component therefore keeps its slot,
// which encodes its initial label (address, bus word), and is one of
//   tier 1: no jump has touched its routing.  Its excited sites are the
//           schedule positions of its live tokens on its own path, so its
//           state changes only at slices whose joint outcome J is nonempty
//           (a lost data token).  Its exposure, sign and weight follow from
//           prefix tables of the schedule.
//   tier 2: a jump removed an address token or a router.  The component
//           follows the gates literally on an explicit site list in a
//           per-workgroup pool (qubit: one list per address, shared by its
//           bus words); short lists are processed in registers, longer ones
//           in global memory.
// Amplitudes are c_i * sign * gamma^{|J|/2} * a^e.  gamma^{|J|/2} is the same
// for every survivor and cancels in every ratio, so a draw uses the weights
// (1-gamma)^e.  Per slice the kernel tests the slice's candidates against
// every component; weights are formed only when some component is hit.
#include "qram_device.h"
#include "qram_records.h"

#include <algorithm>

namespace qr {

// Optional phase timers (build with -DQR_PHASE_TIMERS): wave 0 of every
// workgroup adds the shader-clock cycles spent in each phase of the kernel.
#ifdef QR_PHASE_TIMERS
__device__ unsigned long long qr_phase_cycles[16];
#define QR_TINIT unsigned long long qr_ph[8] = {0, 0, 0, 0, 0, 0, 0, 0}, qr_pn[8] = {0, 0, 0, 0, 0, 0, 0, 0}; \
  unsigned long long qr_t = clock64();
#define QR_TM(i)                               \
  do {                                         \
    const unsigned long long qr_n = clock64(); \
    qr_ph[i] += qr_n - qr_t;                   \
    qr_pn[i] += 1;                             \
    qr_t = qr_n;                               \
  } while (0)
#define QR_TFLUSH                                                   \
  if (threadIdx.x == 0)                                             \
    for (int i = 0; i < 8; ++i) {                                   \
      atomicAdd(&qr_phase_cycles[i], qr_ph[i]);                     \
      atomicAdd(&qr_phase_cycles[8 + i], qr_pn[i]);                 \
    }
#else
#define QR_TINIT
#define QR_TM(i) \
  do {           \
  } while (0)
#define QR_TFLUSH
#endif

namespace {

constexpr uint32_t EMPTY = 0xFFFFu;

// ---------------------------------------------------------------------------
// tier 1
// ---------------------------------------------------------------------------

// Level of site q (0 ground; 1 excited / L; 2 R) of a tier-1 component of
// address a with live data tokens `live` after the gates of slice s.
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

// Site of token tk (address token t < n, data token n + b) of address a
// after the gates of slice s, or -1 outside the tree.
__device__ __forceinline__ int t1_site(const Tables *__restrict__ tb, int s,
                                       uint32_t a, int tk) {
  const uint8_t ps = tb->pos[s][tk];
  if (ps == NONE) return -1;
  const int l = ps >> 1, slot = ps & 1;
  const uint32_t v = (1u << l) - 1u + (a >> (tb->n - l));
  return (int)(2 * v + slot);
}

// Initial state word of the component (address a, bus word b): live tokens =
// the bus word (qubit) or every data bit (qutrit); the qubit sign already
// holds every fetch phase its live tokens will pick up.
template <int ENC>
__device__ __forceinline__ uint32_t init_word(uint32_t memw_a, uint32_t b, uint32_t kmask) {
  const uint32_t live = ENC == QUBIT ? b : kmask;
  const bool sg = ENC == QUBIT && (__popc(live & memw_a & kmask) & 1);
  return W_ALIVE | (live << W_LIVE_SH) | (sg ? W_SIGN : 0u);
}

// Bit b set for every b that is a subset of c (c below 2^k).
__device__ __forceinline__ uint64_t subsets_of(uint32_t c, int k) {
  uint64_t m = 1;
  for (int i = 0; i < k; ++i)
    if ((c >> i) & 1u) m |= m << (1u << i);
  return m;
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

// Candidates of slice s on the path of address a: `ah` when a candidate sits
// on a site every tier-1 component of a excites (an address token of a), `dh`
// the data tokens sitting on candidate sites.
template <int ENC>
__device__ __forceinline__ void t1_addr_hits(const Tables *__restrict__ tb,
                                             int s, uint32_t a, bool big,
                                             int nc, const uint32_t *cdec,
                                             const uint32_t *cbm, bool &ah,
                                             uint32_t &dh) {
  const int n = tb->n;
  ah = false;
  dh = 0;
  if (!big) {
    for (int j = 0; j < nc; ++j) {
      const uint32_t c = cdec[j];
      const uint32_t tk = (c >> 20) & 0xFFu;
      if (tk == NONE) continue;
      const int l = (c >> 16) & 15;
      const uint32_t q = c & 0xFFFFu;
      if ((a >> (n - l)) != (q >> 1) + 1 - (1u << l)) continue;
      if (tk < (uint32_t)n) {
        if ((ENC == QUTRIT && (q & 1u) == 0) || ((a >> (n - 1 - tk)) & 1u)) ah = true;
      } else {
        dh |= 1u << (tk - n);
      }
    }
    return;
  }
  for (int t = 0; t < n; ++t) {
    const uint8_t ps = tb->pos[s][t];
    if (ps == NONE) continue;
    const bool abit = (a >> (n - 1 - t)) & 1u;
    if (!(abit || (ENC == QUTRIT && (ps & 1) == 0))) continue;
    if (cand_bm(cbm, (uint32_t)t1_site(tb, s, a, t))) ah = true;
  }
  for (int b = 0; b < tb->k; ++b) {
    const int q = t1_site(tb, s, a, n + b);
    if (q >= 0 && cand_bm(cbm, (uint32_t)q)) dh |= 1u << b;
  }
}

// Integer exposure through slice s of a tier-1 component (excited sites
// summed over slices 1..s).  wcs: the exposure of each token through slice s
// (address bit p, then data token b), from shared memory.
template <int ENC>
__device__ __forceinline__ uint32_t t1_exposure(const Tables *__restrict__ tb,
                                                const uint8_t *wcs, int s, uint32_t a,
                                                uint32_t dv, uint32_t ek) {
  const int n = tb->n, k = tb->k;
  uint32_t e = ek;
#pragma unroll
  for (int p = 0; p < MAXN; ++p)
    if (p < n && ((a >> p) & 1u)) e += wcs[p];
#pragma unroll
  for (int b = 0; b < MAXK; ++b)
    if (b < k && ((dv >> b) & 1u)) e += wcs[n + b];
  if (ENC == QUTRIT) e += tb->cntR[s];
  return e;
}

// ---------------------------------------------------------------------------
// tier 2, global-memory list (any length)
// ---------------------------------------------------------------------------
template <int ENC>
struct Rec {
  uint16_t *r;
  static constexpr uint32_t SM = ENC == QUTRIT ? 0x7FFFu : 0xFFFFu;
  __device__ __forceinline__ int cnt() const { return r[0]; }
  // a count read back from the pool is trusted up to lmax only
  __device__ __forceinline__ Rec &bound(int lmax, uint32_t *err) {
    if (r[0] > (uint32_t)lmax) {
      flag_err(err, ERR_LIST);
      r[0] = (uint16_t)lmax;
    }
    return *this;
  }
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

// Gates of slice s on a global-memory list (schedule of Sec. II A, gate set
// of App. C; qutrit stores gated by the parent's router).  Returns the sign
// picked up by the qubit fetch.
template <int ENC>
__device__ __attribute__((noinline)) uint32_t t2_gates_mem(const Tables *__restrict__ tb, int s,
                                                           Rec<ENC> R, uint32_t a, uint32_t *err) {
  uint32_t flip = 0;
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
      uint32_t g0 = 0, g1 = 0, g2 = 0, g3 = 0;
      int ng = 0;
      if (sl == 0) {
        ng = 1;
      } else {
        for (int j = 0; j < R.cnt(); ++j) {
          const uint32_t x = R.raw(j), q = x & Rec<ENC>::SM;
          if (q & 1u) continue;
          const uint32_t v = q >> 1;
          if (layer_of(v) != sl - 1) continue;
          const uint32_t c = 2 * v + 1 + ((x & LV_R_BIT) ? 1u : 0u);
          if (ng == 0) g0 = c;
          else if (ng == 1) g1 = c;
          else if (ng == 2) g2 = c;
          else if (ng == 3) g3 = c;
          else atomicOr(err, ERR_LIST);
          ++ng;
        }
      }
      for (int g = 0; g < ng && g < 4; ++g) {
        const uint32_t v = g == 0 ? g0 : g == 1 ? g1 : g == 2 ? g2 : g3;
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
        if ((tb->mem[cell] >> fb) & 1u) flip ^= W_SIGN;
      }
    } else {
      uint32_t c0 = 0, c1 = 0;  // cells' d-site targets of the leaf routers
      int nl = 0;
      for (int j = 0; j < R.cnt(); ++j) {
        const uint32_t x = R.raw(j), q = x & Rec<ENC>::SM;
        if ((q & 1u) || (q >> 1) < v0) continue;
        const uint32_t v = q >> 1;
        const uint32_t cell = 2 * (v - v0) + ((x & LV_R_BIT) ? 1u : 0u);
        const uint32_t tgt = ((tb->mem[cell] >> fb) & 1u) ? 2 * v + 1 : 0xFFFFFFFFu;
        if (nl == 0) c0 = tgt;
        else if (nl == 1) c1 = tgt;
        else atomicOr(err, ERR_LIST);
        ++nl;
      }
      for (int g = 0; g < nl && g < 2; ++g) {
        const uint32_t tgt = g == 0 ? c0 : c1;
        if (tgt != 0xFFFFFFFFu) {
          const uint32_t v = tgt >> 1;
          const int jd = R.find_site(2 * v + 1);
          if (jd >= 0)
            R.remove(jd);
          else if (!R.add(2 * v + 1, lmax))
            atomicOr(err, ERR_LIST);
        }
      }
    }
  }
  return flip;
}

// ---------------------------------------------------------------------------
// tier 2, register list (C entries, empty slots marked)
// ---------------------------------------------------------------------------
template <int ENC, int C>
struct RList {
  // C 16-bit entries, two per register; EMPTY marks a free entry
  uint32_t p[C / 2];
  uint32_t bus;
  bool dirty;  // changed since load: the record needs writing back
  bool holes;  // an entry was removed: the entries may no longer be contiguous
  static constexpr uint32_t SM = ENC == QUTRIT ? 0x7FFFu : 0xFFFFu;

  __device__ __forceinline__ uint32_t get(int j) const {
    return (p[j >> 1] >> ((j & 1) * 16)) & 0xFFFFu;
  }
  __device__ __forceinline__ void set(int j, uint32_t x) {
    const int sh = (j & 1) * 16;
    p[j >> 1] = (p[j >> 1] & ~(0xFFFFu << sh)) | (x << sh);
    dirty = true;
  }
  __device__ __forceinline__ void load(const uint16_t *rec, uint32_t cnt) {
    const uint32_t *r32 = reinterpret_cast<const uint32_t *>(rec);
    bus = r32[0] >> 16;
    dirty = false;
    holes = false;
#pragma unroll
    for (int j = 0; j < C; j += 2) {
      const uint32_t w = (uint32_t)j < cnt ? r32[1 + j / 2] : 0xFFFFFFFFu;
      const uint32_t lo = (uint32_t)j < cnt ? (w & 0xFFFFu) : EMPTY;
      const uint32_t hi = (uint32_t)(j + 1) < cnt ? (w >> 16) : EMPTY;
      p[j >> 1] = lo | (hi << 16);
    }
  }
  // writes at most lim entries (the record's capacity); more raise ovf
  __device__ __forceinline__ uint32_t store(uint16_t *rec, uint32_t lim, bool &ovf) const {
    if (!holes) {  // entries 0 .. cnt-1, empty after: whole words
      uint32_t cnt = 0;
#pragma unroll
      for (int j = 0; j < C; ++j) cnt += get(j) != EMPTY ? 1u : 0u;
      if (cnt > lim) {
        ovf = true;
        cnt = lim;
      }
      uint32_t *r32 = reinterpret_cast<uint32_t *>(rec);
#pragma unroll
      for (int j = 0; j < C; j += 2) {
        if ((uint32_t)j + 1 < cnt)
          r32[1 + j / 2] = p[j >> 1];
        else if ((uint32_t)j < cnt)  // (nothing past the last entry is written)
          rec[2 + j] = (uint16_t)(p[j >> 1] & 0xFFFFu);
      }
      r32[0] = cnt | (bus << 16);
      return cnt;
    }
    uint32_t pos = 0;
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const uint32_t x = get(j);
      if (x != EMPTY) {
        if (pos < lim)
          rec[2 + pos++] = (uint16_t)x;
        else
          ovf = true;
      }
    }
    rec[0] = (uint16_t)pos;
    rec[1] = (uint16_t)bus;
    return pos;
  }
  // (EMPTY & SM is above every site of a tree with n <= 15 (qubit) or
  // n <= 14 (qutrit), so an empty entry never matches a site)
  __device__ __forceinline__ bool has(uint32_t q) const {
    bool f = false;
#pragma unroll
    for (int j = 0; j < C; ++j) f |= (get(j) & SM) == q;
    return f;
  }
  __device__ __forceinline__ void remove_site(uint32_t q) {
#pragma unroll
    for (int j = 0; j < C; ++j)
      if ((get(j) & SM) == q) {
        set(j, EMPTY);
        holes = true;
      }
  }
  __device__ __forceinline__ bool add(uint32_t x) {
    bool placed = false;
#pragma unroll
    for (int j = 0; j < C; ++j)
      if (!placed && get(j) == EMPTY) {
        set(j, x);
        placed = true;
      }
    return placed;
  }
  __device__ __forceinline__ void toggle(uint32_t q, bool &ovf) {
    if (has(q))
      remove_site(q);
    else
      ovf |= !add(q);
  }
  // routing direction of node v: qubit 0/1; qutrit -1 (W), 0 (L), 1 (R)
  __device__ __forceinline__ int dir(uint32_t v) const {
    int d = ENC == QUBIT ? 0 : -1;
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const uint32_t x = get(j);
      if ((x & SM) == 2 * v) d = ENC == QUBIT ? 1 : ((x & LV_R_BIT) ? 1 : 0);
    }
    return d;
  }
  // qutrit store at node v (router site 2v, data site 2v+1): an empty
  // router takes the data site's value (R when it holds one, else L); a set
  // router with an empty data site is unstored (R leaves the data site set).
  // One scan finds both sites, a second applies the change.
  __device__ __forceinline__ void store_node(uint32_t v, bool &ovf) {
    int jr = -1, jd = -1;
    uint32_t xr = 0;
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const uint32_t x = get(j), q = x & SM;
      if (q == 2 * v) {
        jr = j;
        xr = x;
      }
      if (q == 2 * v + 1) jd = j;
    }
    int jsel = -1;
    uint32_t val = 0;
    bool need_add = false;
    if (jr < 0) {
      if (jd >= 0) {
        jsel = jd;
        val = 2 * v | LV_R_BIT;
      } else {
        need_add = true;
        val = 2 * v;
      }
    } else if (jd < 0) {
      jsel = jr;
      val = (xr & LV_R_BIT) ? 2 * v + 1 : EMPTY;
      if (val == EMPTY) holes = true;
    }
    bool placed = false;
#pragma unroll
    for (int j = 0; j < C; ++j) {
      if (j == jsel) {
        set(j, val);
      } else if (need_add && !placed && get(j) == EMPTY) {
        set(j, val);
        placed = true;
      }
    }
    if (need_add && !placed) ovf = true;
  }
  // does a candidate of the slice sit on one of the sites?
  __device__ __forceinline__ bool hit(bool big, int nc, const uint32_t *cdec,
                                      const uint32_t *cbm) const {
    bool h = false;
    if (big) {
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const uint32_t x = get(j);
        if (x != EMPTY) h |= cand_bm(cbm, x & SM);
      }
    } else {
      for (int c = 0; c < nc; ++c) h |= has(cdec[c] & 0xFFFFu);
    }
    return h;
  }
};

template <int ENC, int C>
__device__ __forceinline__ void t2_gates_reg(const Tables *__restrict__ tb, int s,
                                             RList<ENC, C> &L, uint32_t a,
                                             uint32_t &word, bool &ovf) {
  const int n = tb->n;
  constexpr uint32_t SM = RList<ENC, C>::SM;
  const int ct = tb->copy_t[s];
  if (ct >= 0 && ((a >> (n - 1 - ct)) & 1u)) L.toggle(1, ovf);
  const int sl = tb->store_l[s];
  if (sl >= 0) {
    if (ENC == QUBIT) {
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const uint32_t x = L.get(j);
        if (x != EMPTY && layer_of(x >> 1) == sl) L.set(j, x ^ 1u);
      }
    } else {
      uint32_t g0 = 0, g1 = 0, g2 = 0, g3 = 0;
      int ng = 0;
      if (sl == 0) {
        ng = 1;
      } else {
#pragma unroll
        for (int j = 0; j < C; ++j) {
          const uint32_t x = L.get(j);
          if (x == EMPTY || (x & 1u)) continue;
          const uint32_t v = (x & SM) >> 1;
          if (layer_of(v) != sl - 1) continue;
          const uint32_t c = 2 * v + 1 + ((x & LV_R_BIT) ? 1u : 0u);
          if (ng == 0) g0 = c;
          else if (ng == 1) g1 = c;
          else if (ng == 2) g2 = c;
          else if (ng == 3) g3 = c;
          else ovf = true;
          ++ng;
        }
      }
      for (int g = 0; g < 4; ++g) {
        if (g >= ng) break;
        L.store_node(g == 0 ? g0 : g == 1 ? g1 : g == 2 ? g2 : g3, ovf);
      }
    }
  }
  const uint32_t cm = tb->cswap[s];
  if (cm) {
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const uint32_t x = L.get(j);
      if (x == EMPTY || !(x & 1u)) continue;
      const uint32_t v = (x & SM) >> 1;
      const int l = layer_of(v);
      if ((cm >> l) & 1u) {
        const int d = L.dir(v);
        if (d >= 0) L.set(j, 2 * (2 * v + 1 + (uint32_t)d) + 1);
      } else if (l >= 1 && ((cm >> (l - 1)) & 1u)) {
        const uint32_t p = (v - 1) >> 1;
        const int d = L.dir(p);
        if (d >= 0 && v == 2 * p + 1 + (uint32_t)d) L.set(j, 2 * p + 1);
      }
    }
  }
  const int bb = tb->bus_b[s];
  if (bb >= 0) {
    const bool d0 = L.has(1);
    const bool bbit = (L.bus >> bb) & 1u;
    if (d0 && !bbit) {
      L.remove_site(1);
      L.bus |= 1u << bb;
      L.dirty = true;
    } else if (!d0 && bbit) {
      ovf |= !L.add(1);
      L.bus &= ~(1u << bb);
      L.dirty = true;
    }
  }
  const int fb = tb->fetch_b[s];
  if (fb >= 0) {
    const uint32_t v0 = (1u << (n - 1)) - 1u;
    if (ENC == QUBIT) {
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const uint32_t x = L.get(j);
        if (x == EMPTY || !(x & 1u) || (x >> 1) < v0) continue;
        const uint32_t v = x >> 1, p = v - v0;
        if ((tb->mem[2 * p + (uint32_t)L.dir(v)] >> fb) & 1u) word ^= W_SIGN;
      }
    } else {
      uint32_t c0 = 0, c1 = 0;
      int nl = 0;
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const uint32_t x = L.get(j);
        if (x == EMPTY || (x & 1u) || ((x & SM) >> 1) < v0) continue;
        const uint32_t v = (x & SM) >> 1;
        const uint32_t cell = 2 * (v - v0) + ((x & LV_R_BIT) ? 1u : 0u);
        const uint32_t target = (tb->mem[cell] >> fb) & 1u ? 2 * v + 1 : EMPTY;
        if (nl == 0) c0 = target;
        else if (nl == 1) c1 = target;
        else ovf = true;
        ++nl;
      }
      if (nl > 0 && c0 != EMPTY) L.toggle(c0, ovf);
      if (nl > 1 && c1 != EMPTY) L.toggle(c1, ovf);
    }
  }
}

// Gates of slice s on one tier-2 component whose record holds cnt0 entries;
// returns the new count and whether a candidate of the slice sits on one of
// its sites.  Short lists run in registers, long ones in global memory.
template <int ENC>
__device__ __forceinline__ uint32_t t2_step(const Tables *__restrict__ tb,
                                            int s, uint16_t *recp,
                                            uint32_t cnt0, uint32_t a,
                                            uint32_t &word, bool slow, bool big,
                                            int nc, const uint32_t *cdec,
                                            const uint32_t *cbm, bool &hit,
                                            uint32_t &bus, uint32_t *err) {
  // register capacities; the gates of one slice add at most `grow` entries
  constexpr uint32_t C1 = ENC == QUBIT ? 16 : 24, C2 = ENC == QUBIT ? 24 : 32;
  constexpr uint32_t grow = ENC == QUBIT ? 2 : 8;
  bool ovf = false;
  uint32_t cnt;
  hit = false;
  if (!slow && cnt0 + grow <= C1) {
    RList<ENC, C1> L;
    L.load(recp, cnt0);
    t2_gates_reg<ENC, C1>(tb, s, L, a, word, ovf);
    if (nc > 0) hit = L.hit(big, nc, cdec, cbm);
    cnt = L.dirty ? L.store(recp, (uint32_t)tb->lmax, ovf) : cnt0;
    bus = L.bus;
  } else if (!slow && cnt0 + grow <= C2) {
    RList<ENC, C2> L;
    L.load(recp, cnt0);
    t2_gates_reg<ENC, C2>(tb, s, L, a, word, ovf);
    if (nc > 0) hit = L.hit(big, nc, cdec, cbm);
    cnt = L.dirty ? L.store(recp, (uint32_t)tb->lmax, ovf) : cnt0;
    bus = L.bus;
  } else {
    Rec<ENC> R{recp};
    R.bound(tb->lmax, err);
    word ^= t2_gates_mem<ENC>(tb, s, R, a, err);
    cnt = R.cnt();
    bus = R.r[1];
    if (nc > 0)
      for (uint32_t q = 0; q < cnt && !hit; ++q)
        hit = big ? cand_bm(cbm, R.site(q)) : cand_list(cdec, nc, R.site(q));
  }
  if (ovf) atomicOr(err, ERR_LIST);
  return cnt;
}

// Qubit tier 2, shared lists.  Routers and address tokens do not depend on
// the bus word, so the bus words of one address follow the same gates on
// the same routing as long as no gate acts on a data token in a way that
// depends on which bus words carry it.  Such bus words keep one list: the
// address entries (routers, address tokens in transit, residues) as an
// ordinary list, and the site of each data token they may carry, tagged by
// the token.  Record: [0] address entries, [1] bus mask | tagged tokens << 8,
// [2 ..] address entries, [2 + lmax + t] site of tagged token t (EMPTY: on
// the bus or lost), [2 + lmax + k] the split set D.  Bus word b carries the
// tagged tokens b & tokens.
// A store that would move a tagged token into a router makes the bus words
// that carry it route differently from those that do not, so before such a
// store every class splits on the tokens concerned: the bus words of an
// address fall into classes c (a subset of D) of the b with b & D = c, each
// with its own list in the record slot of bus word c; in class c the tokens
// of D are untagged, entries of the list when c holds them, gone otherwise.
// Any other gate that would treat a class's bus words differently (rare)
// turns the class into one ordinary list per component (state bit W_SPLIT).
constexpr int QK = 6;  // data tokens of the qubit encoding at most

struct TokPos {
  // two 16-bit sites per register; a runtime token number selects among the
  // registers (no indexed array, which would live in scratch memory)
  uint32_t p[QK / 2];
  __device__ __forceinline__ uint32_t word(int t) const { return t < 2 ? p[0] : (t < 4 ? p[1] : p[2]); }
  __device__ __forceinline__ uint32_t get(int t) const { return (word(t) >> ((t & 1) * 16)) & 0xFFFFu; }
  __device__ __forceinline__ void set(int t, uint32_t x) {
    const int sh = (t & 1) * 16;
    const uint32_t w = (word(t) & ~(0xFFFFu << sh)) | (x << sh);
    p[0] = t < 2 ? w : p[0];
    p[1] = (t >= 2 && t < 4) ? w : p[1];
    p[2] = t >= 4 ? w : p[2];
  }
  __device__ __forceinline__ void load(const uint16_t *r, int k) {
#pragma unroll
    for (int t = 0; t < QK; t += 2) {
      const uint32_t lo = t < k ? (uint32_t)r[t] : EMPTY;
      const uint32_t hi = t + 1 < k ? (uint32_t)r[t + 1] : EMPTY;
      p[t >> 1] = lo | (hi << 16);
    }
  }
  __device__ __forceinline__ void store(uint16_t *r, int k) const {
#pragma unroll
    for (int t = 0; t < QK; ++t)
      if (t < k) r[t] = (uint16_t)get(t);
  }
  // data token at site q, or -1
  __device__ __forceinline__ int at(uint32_t q) const {
    int r = -1;
#pragma unroll
    for (int t = 0; t < QK; ++t)
      if (get(t) == q) r = t;
    return r;
  }
};

// Gates of slice s (same order and rules as t2_gates_reg) on a shared list.
// Returns false as soon as a gate would act differently on bus words that
// carry different tokens; the caller then discards the registers.
template <int C>
__device__ __forceinline__ bool t2_gates_shared(const Tables *__restrict__ tb, int s,
                                                RList<QUBIT, C> &L, TokPos &tp, uint32_t a,
                                                uint32_t toks, uint32_t &busm, bool &flip_all,
                                                uint32_t &flip_tok, bool &moved, bool &ovf) {
  const int n = tb->n;
  const int ct = tb->copy_t[s];
  if (ct >= 0 && ((a >> (n - 1 - ct)) & 1u)) {
    if (tp.at(1) >= 0) return false;
    L.toggle(1, ovf);
  }
  const int sl = tb->store_l[s];
  if (sl >= 0) {
#pragma unroll
    for (int t = 0; t < QK; ++t) {
      const uint32_t x = tp.get(t);
      if (x != EMPTY && layer_of(x >> 1) == sl) return false;
    }
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const uint32_t x = L.get(j);
      if (x != EMPTY && layer_of(x >> 1) == sl) L.set(j, x ^ 1u);
    }
  }
  const uint32_t cm = tb->cswap[s];
  if (cm) {
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const uint32_t x = L.get(j);
      if (x == EMPTY || !(x & 1u)) continue;
      const uint32_t v = x >> 1;
      const int l = layer_of(v);
      if ((cm >> l) & 1u) {
        L.set(j, 2 * (2 * v + 1 + (uint32_t)L.dir(v)) + 1);
      } else if (l >= 1 && ((cm >> (l - 1)) & 1u)) {
        const uint32_t p = (v - 1) >> 1;
        if (v == 2 * p + 1 + (uint32_t)L.dir(p)) L.set(j, 2 * p + 1);
      }
    }
#pragma unroll
    for (int t = 0; t < QK; ++t) {
      const uint32_t x = tp.get(t);
      if (x == EMPTY) continue;
      const uint32_t v = x >> 1;
      const int l = layer_of(v);
      if ((cm >> l) & 1u) {
        tp.set(t, 2 * (2 * v + 1 + (uint32_t)L.dir(v)) + 1);
        moved = true;
      } else if (l >= 1 && ((cm >> (l - 1)) & 1u)) {
        const uint32_t p = (v - 1) >> 1;
        if (v == 2 * p + 1 + (uint32_t)L.dir(p)) {
          tp.set(t, 2 * p + 1);
          moved = true;
        }
      }
    }
  }
  const int bb = tb->bus_b[s];
  if (bb >= 0) {
    const int t1 = tp.at(1);
    if ((toks >> bb) & 1u) {  // the bus qubit's own token is tagged
      if (L.has(1) || (t1 >= 0 && t1 != bb)) return false;
      if (t1 == bb) {
        tp.set(bb, EMPTY);
        busm |= 1u << bb;
        moved = true;
      } else if ((busm >> bb) & 1u) {
        tp.set(bb, 1);
        busm &= ~(1u << bb);
        moved = true;
      }
    } else {  // untagged: the bus qubit is the same in every bus word of the list
      if (t1 >= 0) return false;
      const bool d0 = L.has(1), bbit = (busm >> bb) & 1u;
      if (d0 && !bbit) {
        L.remove_site(1);
        busm |= 1u << bb;
      } else if (!d0 && bbit) {
        ovf |= !L.add(1);
        busm &= ~(1u << bb);
      }
    }
  }
  const int fb = tb->fetch_b[s];
  if (fb >= 0) {
    const uint32_t v0 = (1u << (n - 1)) - 1u;
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const uint32_t x = L.get(j);
      if (x == EMPTY || !(x & 1u) || (x >> 1) < v0) continue;
      const uint32_t v = x >> 1;
      if ((tb->mem[2 * (v - v0) + (uint32_t)L.dir(v)] >> fb) & 1u) flip_all = !flip_all;
    }
#pragma unroll
    for (int t = 0; t < QK; ++t) {
      const uint32_t x = tp.get(t);
      if (x == EMPTY || (x >> 1) < v0) continue;
      const uint32_t v = x >> 1;
      if ((tb->mem[2 * (v - v0) + (uint32_t)L.dir(v)] >> fb) & 1u) flip_tok ^= 1u << t;
    }
  }
  return true;
}

// One slice on a shared list held in registers (C entries).  Returns false,
// with nothing written, when the address has to split first.
template <int C>
__device__ __forceinline__ bool t2_shared_reg(const Tables *__restrict__ tb, int s, uint16_t *recp,
                                              uint32_t cnt0, uint32_t a, bool big, int nc,
                                              const uint32_t *cdec, const uint32_t *cbm,
                                              uint32_t &cnt, uint32_t &busf, bool &flip_all,
                                              uint32_t &flip_tok, bool &hit_all, uint32_t &hit_tok,
                                              bool &split_next, uint32_t *err) {
  const int k = tb->k;
  RList<QUBIT, C> L;
  L.load(recp, cnt0);
  TokPos tp;
  tp.load(recp + 2 + tb->lmax, k);
  uint32_t busm = L.bus & 0xFFu;
  bool moved = false, ovf = false;
  if (!t2_gates_shared<C>(tb, s, L, tp, a, (L.bus >> 8) & 0xFFu, busm, flip_all, flip_tok, moved, ovf))
    return false;
  if (ovf) atomicOr(err, ERR_LIST);
  if (busm != (L.bus & 0xFFu)) {
    L.bus = (L.bus & 0xFF00u) | busm;
    L.dirty = true;
  }
  if (nc > 0) {
    if (big) {
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const uint32_t x = L.get(j);
        if (x != EMPTY && cand_bm(cbm, x)) hit_all = true;
      }
#pragma unroll
      for (int t = 0; t < QK; ++t) {
        const uint32_t x = tp.get(t);
        if (x != EMPTY && cand_bm(cbm, x)) hit_tok |= 1u << t;
      }
    } else {
      for (int c = 0; c < nc; ++c) {
        const uint32_t q = cdec[c] & 0xFFFFu;
        if (L.has(q)) hit_all = true;
        const int t = tp.at(q);
        if (t >= 0) hit_tok |= 1u << t;
      }
    }
  }
  bool sovf = false;
  cnt = L.dirty ? L.store(recp, (uint32_t)tb->lmax, sovf) : cnt0;
  if (sovf) atomicOr(err, ERR_LIST);
  if (moved) tp.store(recp + 2 + tb->lmax, k);
  busf = L.bus;
  // a tagged token on the store layer of the next slice: the class must be
  // split before that store
  split_next = false;
  if (s + 1 < tb->T && tb->store_l[s + 1] >= 0) {
    const int nsl = tb->store_l[s + 1];
    const uint32_t toks = (L.bus >> 8) & 0xFFu;
#pragma unroll
    for (int t = 0; t < QK; ++t) {
      const uint32_t x = tp.get(t);
      if (((toks >> t) & 1u) && x != EMPTY && layer_of(x >> 1) == nsl) split_next = true;
    }
  }
  return true;
}

// Tagged tokens that the store of slice s would move into a router, over
// the classes cl of the address whose class-0 record is r0.
__device__ __forceinline__ uint32_t class_store_tokens(const Tables *__restrict__ tb, int s,
                                                       const uint16_t *r0, int rec, uint64_t cl) {
  const int sl = tb->store_l[s], k = tb->k, lmax = tb->lmax;
  uint32_t X = 0;
  for (uint64_t m = cl; m; m &= m - 1) {
    const uint16_t *rc = r0 + (size_t)(__ffsll((unsigned long long)m) - 1) * rec;
    const uint32_t toks = ((uint32_t)rc[1] >> 8) & 0xFFu;
    for (int t = 0; t < k; ++t) {
      const uint32_t x = rc[2 + lmax + t];
      if (((toks >> t) & 1u) && x != EMPTY && layer_of(x >> 1) == sl) X |= 1u << t;
    }
  }
  return X;
}

// ---------------------------------------------------------------------------
// shared memory layout
// ---------------------------------------------------------------------------
__host__ __device__ inline uint32_t al16(uint32_t x) { return (x + 15u) & ~15u; }

struct Sm {
  double *red;      // [2 * nw * 8]
  double *scanb;    // [nw]
  double *fw;       // factor tables (1-gamma)^m: A chunks [3*32], data [256], lost [256]
  double *fa;       // the same with a^m (final)
  double *fmisc;    // [4]
  uint32_t *cstart; // [MAXT + 1] first candidate of each slice
  uint8_t *nxt;     // [MAXT + 1] first slice >= s holding a candidate (T: none)
  uint32_t *cdec;   // [cdec_cap]: the slice's decoded candidates, or all of them
  uint32_t *Jb;     // [JMAX]
  int *misc;        // [8]
  uint32_t *cbm;    // [(M + 31) / 32]
  uint32_t *badl;   // [(D + 31) / 32]
  uint8_t *wc;      // [T * (n + k)] exposure counts of each token through each slice
  uint32_t *st;     // [e_cap] when the state lives in LDS
};

constexpr int F_A = 0, F_D = 96, F_K = 96 + 256, F_N = 96 + 256 + 256;

__host__ __device__ inline uint32_t fixed_bytes(int M, int D, int threads, uint32_t cdec_cap,
                                                uint32_t walk_bytes) {
  const int nw = threads >> 6;
  uint32_t b = 0;
  b += al16(2 * nw * 8 * 8);
  b += al16(nw * 8);
  b += al16(F_N * 8) * 2;
  b += al16(4 * 8);
  b += al16((MAXT + 1) * 4);
  b += al16(MAXT + 1);
  b += al16(cdec_cap * 4);
  b += al16(JMAX * 4);
  b += al16(8 * 4);
  b += al16(((M + 31) / 32) * 4);
  b += al16(((D + 31) / 32) * 4);
  b += al16(walk_bytes);
  return b;
}

__device__ inline Sm carve(unsigned char *base, int M, int D, int threads, uint32_t cdec_cap,
                           uint32_t walk_bytes) {
  const int nw = threads >> 6;
  Sm m;
  unsigned char *p = base;
  m.red = reinterpret_cast<double *>(p);
  p += al16(2 * nw * 8 * 8);
  m.scanb = reinterpret_cast<double *>(p);
  p += al16(nw * 8);
  m.fw = reinterpret_cast<double *>(p);
  p += al16(F_N * 8);
  m.fa = reinterpret_cast<double *>(p);
  p += al16(F_N * 8);
  m.fmisc = reinterpret_cast<double *>(p);
  p += al16(4 * 8);
  m.cstart = reinterpret_cast<uint32_t *>(p);
  p += al16((MAXT + 1) * 4);
  m.nxt = reinterpret_cast<uint8_t *>(p);
  p += al16(MAXT + 1);
  m.cdec = reinterpret_cast<uint32_t *>(p);
  p += al16(cdec_cap * 4);
  m.Jb = reinterpret_cast<uint32_t *>(p);
  p += al16(JMAX * 4);
  m.misc = reinterpret_cast<int *>(p);
  p += al16(8 * 4);
  m.cbm = reinterpret_cast<uint32_t *>(p);
  p += al16(((M + 31) / 32) * 4);
  m.badl = reinterpret_cast<uint32_t *>(p);
  p += al16(((D + 31) / 32) * 4);
  m.wc = reinterpret_cast<uint8_t *>(p);
  p += al16(walk_bytes);
  m.st = reinterpret_cast<uint32_t *>(p);
  return m;
}

// Factor tables of slice s into shared memory: (1-gamma)^e or a^e of the
// exposure through slice s for the three 5-bit chunks of the address bits
// (bit n-1-t is address token t), for every data-token set, and the router
// factor (qutrit).  The host precomputes them per slice.
template <int ENC>
__device__ __forceinline__ void load_factors(const Tables *__restrict__ tb, int s,
                                             const double *__restrict__ ftab, double *f,
                                             double *fmisc) {
  const int nd = 1 << tb->k, nfs = tb->nfs;
  const double *__restrict__ src = ftab + (size_t)s * nfs;
  for (int x = threadIdx.x; x < F_D + nd; x += blockDim.x) f[x] = src[x];  // F_A = 0, F_D = 96
  if (threadIdx.x == 0) *fmisc = ENC == QUTRIT ? src[F_D + nd] : 1.0;
}

// Exposure factors of data tokens lost to jumps (index = exposure).
__device__ __forceinline__ void load_lost(const Tables *__restrict__ tb,
                                          const double *__restrict__ pw, double *f) {
  const int kmax = min(255, tb->emax);
  for (int m = threadIdx.x; m <= kmax; m += blockDim.x) f[F_K + m] = pw[m];
}

__device__ __forceinline__ double fA(const double *f, uint32_t a) {
  return f[F_A + (a & 31u)] * f[F_A + 32 + ((a >> 5) & 31u)] * f[F_A + 64 + ((a >> 10) & 31u)];
}

// ---------------------------------------------------------------------------
// qubit: slices before the first jump, one wave
// ---------------------------------------------------------------------------
constexpr int WALK_MAXC = 6;   // token candidates per slice the walk combines
constexpr int WALK_MAXA = 64;  // qutrit: addresses per slice the walk sums over

// Until the first jump every component keeps its initial label: address a
// and bus word b (qubit) or the fetched data bits (qutrit).  A candidate on
// a token site then hits the components whose address lies below its node
// (fixed leading address bits) and whose token there is excited: one more
// address bit set, or, for a data token, one bus bit set (qubit) or that
// memory bit fetched (qutrit).  Good branches are never hit, so the sum of
// the weights of the hit components over every address equals the sum over
// the explicit ones, and with the slice's closed-form total it decides the
// slice's draw (Eq. maskweight) as the block does, without a pass over the
// components.  The draws of different slices are independent until the
// first jump, so each thread of the block takes one slice.
//   qubit: the weight before the layer of slice s factorises over the
//     tokens, the product of f_p = (1-gamma)^e over the set address bits p
//     and of g_c over the set bus bits c (e: that token's exposure through
//     slice s-1).  An intersection of hit sets fixes some address and bus
//     bits, so its weight is a product, and the weight of the union follows
//     by inclusion-exclusion over the slice's token candidates.
//   qutrit: the data factor depends on the memory word, so the thread sums
//     the weights of the hit addresses over the union of the candidates'
//     subtrees (nested subtrees taken once).
//
// Does slice s need the block: does its draw pick a nonempty J, or has it
// more candidates (or, qutrit, addresses to sum) than one thread combines?
template <int ENC>
__device__ __forceinline__ bool nojump_stop(const Tables *__restrict__ tb, const Run *rp,
                                            const Sm &sm, const uint32_t *__restrict__ cand,
                                            bool pre, int s, uint32_t traj) {
  const int n = tb->n, k = tb->k, nb = n + k;
  const uint32_t cb = sm.cstart[s];
  const int nc = (int)(sm.cstart[s + 1] - cb);
  if (nc == 0) return false;
  if (nc > NCS) return true;
  // the slice's token candidates, decoded: site | layer << 16 | token << 20
  uint32_t cq[WALK_MAXC];
  int m = 0;
  for (int c = 0; c < nc; ++c) {
    uint32_t x;
    if (pre) {
      x = sm.cdec[cb + c];
    } else {
      const uint32_t q = cand[cb + c] - (uint32_t)(s - 1) * (uint32_t)tb->M;
      const int l = layer_of(q >> 1);
      x = q | ((uint32_t)l << 16) | ((uint32_t)tb->tok[s][l][q & 1u] << 20);
    }
    if (((x >> 20) & 0xFFu) == NONE) continue;
    if (m == WALK_MAXC) return true;
#pragma unroll
    for (int i = 0; i < WALK_MAXC; ++i)
      if (i == m) cq[i] = x;
    ++m;
  }
  if (m == 0) return false;
  const uint8_t *wc = sm.wc + (s - 1) * nb;  // exposure of each token through slice s-1
  double H = 0.0;
  if (ENC == QUBIT) {
    for (uint32_t S = 1; S < (1u << m); ++S) {
      // the subset S: address bits forced to 1 / to 0, bus bits forced to 1
      uint32_t a1 = 0, a0 = 0, b1 = 0;
#pragma unroll
      for (int i = 0; i < WALK_MAXC; ++i) {
        if (!((S >> i) & 1u)) continue;
        const uint32_t x = cq[i], tk = (x >> 20) & 0xFFu;
        const int l = (int)((x >> 16) & 15u);
        const uint32_t idx = ((x & 0xFFFFu) >> 1) + 1u - (1u << l);
        const uint32_t one = idx << (n - l);
        a1 |= one;
        a0 |= (((1u << l) - 1u) << (n - l)) & ~one;
        if (tk < (uint32_t)n)
          a1 |= 1u << (n - 1 - (int)tk);
        else
          b1 |= 1u << (tk - (uint32_t)n);
      }
      if (a1 & a0) continue;
      double w = 1.0;
      for (int p = 0; p < nb; ++p) {
        const double f = sm.fw[F_K + wc[p]];
        const bool one = p < n ? ((a1 >> p) & 1u) : ((b1 >> (p - n)) & 1u);
        const bool zero = p < n && ((a0 >> p) & 1u);
        w *= one ? f : (zero ? 1.0 : 1.0 + f);
      }
      H += (__popc(S) & 1) ? w : -w;
    }
  } else {
    // each hit-capable candidate: subtree [lo, lo + len) and what it needs
    // there: 1 nothing (a stored router), 2 address bit cbit set, 3 memory
    // bit cbit fetched
    uint32_t lo[WALK_MAXC], len[WALK_MAXC], cond[WALK_MAXC], cbit[WALK_MAXC];
#pragma unroll
    for (int i = 0; i < WALK_MAXC; ++i) {
      lo[i] = len[i] = cond[i] = cbit[i] = 0;
      if (i >= m) continue;
      const uint32_t x = cq[i], tk = (x >> 20) & 0xFFu;
      const int l = (int)((x >> 16) & 15u);
      lo[i] = (((x & 0xFFFFu) >> 1) + 1u - (1u << l)) << (n - l);
      len[i] = 1u << (n - l);
      if (tk < (uint32_t)n) {
        cond[i] = (x & 1u) ? 2u : 1u;
        cbit[i] = (uint32_t)(n - 1) - tk;
      } else {
        cbit[i] = tk - (uint32_t)n;
        cond[i] = ((tb->dmask[s] >> cbit[i]) & 1u) ? 3u : 0u;
      }
    }
    // subtrees to sum over: inside no other one (equal ones: the first)
    uint32_t outer = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < WALK_MAXC; ++i) {
      if (!cond[i]) continue;
      bool inner = false;
#pragma unroll
      for (int j = 0; j < WALK_MAXC; ++j)
        if (j != i && cond[j] && lo[i] >= lo[j] && lo[i] + len[i] <= lo[j] + len[j] &&
            (len[i] < len[j] || lo[i] != lo[j] || j < i))
          inner = true;
      if (!inner) {
        outer |= 1u << i;
        tot += len[i];
      }
    }
    if (tot > (uint32_t)WALK_MAXA) return true;
    if (outer) {
      const uint32_t kmask = (1u << k) - 1u;
      const double wr = tb->ftab_w[(size_t)(s - 1) * tb->nfs + F_D + (1 << k)];  // router factor
#pragma unroll
      for (int e = 0; e < WALK_MAXC; ++e) {
        if (!((outer >> e) & 1u)) continue;
        for (uint32_t a = lo[e]; a < lo[e] + len[e]; ++a) {
          const uint32_t memw = tb->mem[a];
          bool hit = false;
#pragma unroll
          for (int c = 0; c < WALK_MAXC; ++c) {
            const bool ok = cond[c] == 1u || (cond[c] == 2u && ((a >> cbit[c]) & 1u)) ||
                            (cond[c] == 3u && ((memw >> cbit[c]) & 1u));
            hit |= cond[c] && (a - lo[c]) < len[c] && ok;
          }
          if (!hit) continue;
          double w = wr;
          for (int p = 0; p < n; ++p)
            if ((a >> p) & 1u) w *= sm.fw[F_K + wc[p]];
          const uint32_t dv = memw & kmask;
          for (int c = 0; c < k; ++c)
            if ((dv >> c) & 1u) w *= sm.fw[F_K + wc[n + c]];
          H += w;
        }
      }
    }
  }
  if (!(H > 0.0)) return false;
  const double u = rp->forced ? rp->uaux[s] : uniform53(rp->seed, (uint32_t)s, 0, traj, 2u);
  const double wall = tb->ctot[s - 1];
  return !(u * wall < wall - H);
}

// The first slice from s0 on that the block must evolve (T: none), every
// slice decided by one thread.  Called by every thread of the block.
template <int ENC>
__device__ __forceinline__ int nojump_walk(const Tables *__restrict__ tb, const Run *rp,
                                           const Sm &sm, const uint32_t *__restrict__ cand,
                                           bool pre, int s0, uint32_t traj) {
  const int T = tb->T;
  const int nw = (int)(blockDim.x >> 6), wave = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
  int *wmin = reinterpret_cast<int *>(sm.scanb);
  for (int base = s0; base < T; base += (int)blockDim.x) {
    const int s = base + (int)threadIdx.x;
    const bool stop = s < T && nojump_stop<ENC>(tb, rp, sm, cand, pre, s, traj);
    const uint64_t bal = __ballot(stop);
    if (lane == 0) wmin[wave] = bal ? base + (wave << 6) + (__ffsll((unsigned long long)bal) - 1) : T;
    __syncthreads();
    int r = T;
    for (int w = 0; w < nw; ++w) r = min(r, wmin[w]);
    if (r < T) return r;
    __syncthreads();
  }
  return T;
}

__device__ __forceinline__ double readlane_f64(double x, int l) {
  const uint64_t b = (uint64_t)__double_as_longlong(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

constexpr int WAVE_MAXA = 2048;  // addresses per slice the wave sums over

// Qutrit, the same walk with the 64 lanes of a wave on one slice at a time
// (qutrit workgroups are small, and the lanes share a slice's subtrees).
// Wave w of nw takes the w-th, (w+nw)-th, ... slice with candidates from s
// on; returns the first of its slices the block must evolve, or T.
template <int ENC>
__device__ __forceinline__ int nojump_walk_wave(const Tables *__restrict__ tb, const Run *rp,
                                                const Sm &sm, const uint32_t *__restrict__ cand,
                                                bool pre, int s, uint32_t traj, int w, int nw) {
  const int n = tb->n, k = tb->k, T = tb->T, nb = n + k;
  const uint32_t M = (uint32_t)tb->M;
  const uint32_t kmask = (1u << k) - 1u;
  const int lane = threadIdx.x & 63;
  for (int i = 0; i < w && s < T; ++i) s = sm.nxt[s + 1];
  while (s < T) {
    const uint32_t cb = sm.cstart[s];
    const int nc = (int)(sm.cstart[s + 1] - cb);
    if (nc > NCS) return s;
    uint32_t x = 0;
    if (lane < nc) {
      if (pre) {
        x = sm.cdec[cb + lane];
      } else {
        const uint32_t q = cand[cb + lane] - (uint32_t)(s - 1) * M;
        const int l = layer_of(q >> 1);
        x = q | ((uint32_t)l << 16) | ((uint32_t)tb->tok[s][l][q & 1u] << 20);
      }
    }
    const uint32_t tk = (x >> 20) & 0xFFu;
    const int l = (int)((x >> 16) & 15u);
    const uint32_t idx = ((x & 0xFFFFu) >> 1) + 1u - (1u << l);  // node's index in its layer
    // lane p < n: f_p; lane n + c: g_c (slice s-1)
    double f = 1.0;
    if (lane < nb) f = sm.fw[F_K + sm.wc[(s - 1) * nb + lane]];
    double H = 0.0;
    {
      // this lane's candidate: subtree [lo, lo + len) and what it needs to be
      // excited there: 1 always (a stored router), 2 address bit cbit set,
      // 3 memory bit cbit fetched
      uint32_t lo = 0, len = 0, cond = 0, cbit = 0;
      if (lane < nc && tk != NONE) {
        lo = idx << (n - l);
        len = 1u << (n - l);
        if (tk < (uint32_t)n) {
          cond = (x & 1u) ? 2u : 1u;
          cbit = (uint32_t)(n - 1) - tk;
        } else {
          cbit = tk - (uint32_t)n;
          cond = ((tb->dmask[s] >> cbit) & 1u) ? 3u : 0u;
        }
      }
      const uint64_t hb = __ballot(cond != 0u);
      const int m = __popcll(hb);
      if (m > WALK_MAXC) return s;
      if (m > 0) {
        // subtrees to sum over: those inside no other one (equal ones: the first)
        bool inner = false;
        for (uint64_t r = hb; r; r &= r - 1) {
          const int src = __ffsll((unsigned long long)r) - 1;
          const uint32_t lo2 = (uint32_t)__builtin_amdgcn_readlane((int)lo, src);
          const uint32_t len2 = (uint32_t)__builtin_amdgcn_readlane((int)len, src);
          if (src != lane && lo >= lo2 && lo + len <= lo2 + len2 && (len < len2 || lo != lo2 || src < lane))
            inner = true;
        }
        const uint64_t eb = __ballot(cond != 0u && !inner);
        uint32_t tot = 0;
        for (uint64_t r = eb; r; r &= r - 1)
          tot += (uint32_t)__builtin_amdgcn_readlane((int)len, __ffsll((unsigned long long)r) - 1);
        if (tot > (uint32_t)WAVE_MAXA) return s;
        const double wr = tb->ftab_w[(size_t)(s - 1) * tb->nfs + F_D + (1 << k)];  // router factor
        double h = 0.0;
        for (uint64_t r = eb; r; r &= r - 1) {
          const int src = __ffsll((unsigned long long)r) - 1;
          const uint32_t lo2 = (uint32_t)__builtin_amdgcn_readlane((int)lo, src);
          const uint32_t len2 = (uint32_t)__builtin_amdgcn_readlane((int)len, src);
          for (uint32_t o = (uint32_t)lane; o < len2; o += 64) {
            const uint32_t a = lo2 + o;
            const uint32_t memw = tb->mem[a];
            bool hit = false;
            for (uint64_t r2 = hb; r2; r2 &= r2 - 1) {
              const int c = __ffsll((unsigned long long)r2) - 1;
              const uint32_t clo = (uint32_t)__builtin_amdgcn_readlane((int)lo, c);
              const uint32_t clen = (uint32_t)__builtin_amdgcn_readlane((int)len, c);
              const uint32_t cc = (uint32_t)__builtin_amdgcn_readlane((int)cond, c);
              const uint32_t cbt = (uint32_t)__builtin_amdgcn_readlane((int)cbit, c);
              const bool ok = cc == 1u || (cc == 2u && ((a >> cbt) & 1u)) || (cc == 3u && ((memw >> cbt) & 1u));
              hit |= (a - clo) < clen && ok;
            }
            if (!hit) continue;
            double w = wr;
            for (int p = 0; p < n; ++p) {
              const double fp = readlane_f64(f, p);
              if ((a >> p) & 1u) w *= fp;
            }
            const uint32_t dv = memw & kmask;
            for (int c = 0; c < k; ++c) {
              const double gc = readlane_f64(f, n + c);
              if ((dv >> c) & 1u) w *= gc;
            }
            h += w;
          }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) h += __shfl_xor(h, off, 64);
        H = readlane_f64(h, 0);
      }
    }
    if (H > 0.0) {
      const double u = rp->forced ? rp->uaux[s] : uniform53(rp->seed, (uint32_t)s, 0, traj, 2u);
      const double wall = tb->ctot[s - 1];
      if (!(u * wall < wall - H)) return s;
    }
    for (int i = 0; i < nw && s < T; ++i) s = sm.nxt[s + 1];
  }
  return T;
}

// ---------------------------------------------------------------------------
// test entry: export of the final pre-measurement components
// ---------------------------------------------------------------------------

// Exposure through the last slice of a component on its no-jump routing:
// address bits of a, carried data tokens dv, lost-token exposure ek.
template <int ENC>
__device__ uint32_t t1_final_exposure(const Tables *__restrict__ tb, uint32_t a, uint32_t dv, uint32_t ek) {
  const int T = tb->T, n = tb->n;
  uint32_t e = ek;
  for (int p = 0; p < n; ++p)
    if ((a >> p) & 1u) e += tb->cntA[T - 1][n - 1 - p];
  for (int b = 0; b < tb->k; ++b)
    if ((dv >> b) & 1u) e += tb->cntD[T - 1][b];
  if (ENC == QUTRIT) e += tb->cntR[T - 1];
  return e;
}

// Record of a component without a site list (ground tree at the end).
template <int ENC>
__device__ void export_ground(const Tables *__restrict__ tb, uint32_t *out, uint32_t a, uint32_t b,
                              uint32_t bus, bool sign, uint32_t e) {
  const int K2 = ENC == QUBIT ? tb->K2 : 1;
  uint32_t *o = out + (size_t)(a * (uint32_t)K2 + b) * (3u + (uint32_t)tb->lmax);
  o[0] = a | (bus << 16) | (sign ? 1u << 24 : 0u) | EXP_PRESENT;
  o[1] = e;
  o[2] = 0;
}

// Record of an explicit component (state word w) of address a (slot g) and
// bus word b after the last slice.
template <int ENC>
__device__ void export_explicit(const Tables *__restrict__ tb, uint32_t *out, const uint16_t *pool, int rec,
                                uint32_t g, uint32_t a, uint32_t b, uint32_t w, uint32_t memw) {
  const int K2 = ENC == QUBIT ? tb->K2 : 1, lmax = tb->lmax, k = tb->k;
  if (!(w & W_DEV)) {
    const uint32_t live = (w >> W_LIVE_SH) & 0xFFu;
    const uint32_t dv = ENC == QUBIT ? live : (live & memw);
    export_ground<ENC>(tb, out, a, b, dv, (w & W_SIGN) != 0, t1_final_exposure<ENC>(tb, a, dv, w & W_EK));
    return;
  }
  uint32_t *o = out + (size_t)(a * (uint32_t)K2 + b) * (3u + (uint32_t)lmax);
  const bool fb = (w & W_FBUS) != 0u;
  const uint32_t cnt = fb ? 0u : (w & W_CNT) >> W_CNT_SH;
  uint32_t bus, m = 0;
  if (fb) {
    bus = (w & W_CNT) >> W_CNT_SH;
  } else if (ENC == QUBIT && !(w & W_SPLIT)) {
    // a shared list: the class's entries plus the tagged tokens b carries
    const uint16_t *r0 = pool + (size_t)g * K2 * rec;
    const uint16_t *rc = r0 + (size_t)(b & r0[2 + lmax + k]) * rec;
    const uint32_t bf = rc[1], toks = (bf >> 8) & 0xFFu;
    bus = bf & (~toks | b) & 0xFFu;
    const uint32_t nc = min((uint32_t)rc[0], (uint32_t)lmax);
    for (uint32_t j = 0; j < nc && m < (uint32_t)lmax; ++j) o[3 + m++] = (uint32_t)rc[2 + j] | (1u << 16);
    for (int t = 0; t < k; ++t) {
      const uint32_t x = rc[2 + lmax + t];
      if (((b & toks) >> t) & 1u && x != EMPTY && m < (uint32_t)lmax) o[3 + m++] = x | (1u << 16);
    }
  } else {
    const uint16_t *r = pool + (size_t)(g * K2 + b) * rec;
    bus = r[1];
    const uint32_t nc = min((uint32_t)r[0], (uint32_t)lmax);
    for (uint32_t j = 0; j < nc; ++j) {
      const uint32_t x = r[2 + j], q = ENC == QUTRIT ? (x & 0x7FFFu) : x;
      const uint32_t lev = (ENC == QUTRIT && (x & LV_R_BIT)) ? 2u : 1u;
      o[3 + m++] = q | (lev << 16);
    }
  }
  if (fb) m = 0;
  (void)cnt;
  o[0] = a | (bus << 16) | ((w & W_SIGN) ? 1u << 24 : 0u) | EXP_PRESENT;
  o[1] = (w & W_E) + cnt;
  o[2] = m;
}

// ---------------------------------------------------------------------------
// the kernel
// ---------------------------------------------------------------------------
template <int ENC, bool SL>
__global__ void __launch_bounds__(ENC == QUBIT ? 1024 : 512) __attribute__((amdgpu_waves_per_eu(ENC == QUBIT ? 4 : 5))) k_evolve(const Tables *__restrict__ tb,
                                                 const Run R_) {
  const Run *rp = &R_;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int n = tb->n, T = tb->T, M = tb->M, D = tb->D, emax = tb->emax;
  const int K2 = ENC == QUBIT ? tb->K2 : 1;
  const int kb = ENC == QUBIT ? tb->k : 0;
  const uint32_t kmask = (1u << tb->k) - 1u;
  const uint64_t kfull = K2 >= 64 ? ~0ull : ((1ull << K2) - 1ull);
  const double *__restrict__ wpow = tb->wpow + emax;
  const double *__restrict__ apow = tb->apow + emax;
  const uint32_t *__restrict__ mem = tb->mem;
  Sm sm = carve(smem, M, D, nthr, rp->cdec_all ? rp->cand_cap : (uint32_t)NCS,
                walk_table_bytes(T, n, tb->k));
  uint32_t *st = SL ? sm.st : rp->gstate + (size_t)blockIdx.x * rp->e_cap;
  const int rec = tb->rec;
  uint16_t *pool = rp->pool + (size_t)blockIdx.x * rp->pool_slots * rec;
  uint32_t *devl = rp->devl + (size_t)blockIdx.x * rp->pool_slots;
  const bool pruned = rp->mode == 1;
  const uint32_t ccap = rp->cand_cap;
  const uint32_t apt = rp->apt;
  const uint32_t bkt = rp->bucket;
  const bool slow_all = rp->tier2_slow != 0;
  const bool pre = rp->cdec_all != 0;  // every candidate decoded into shared memory up front
  int big_prev_s = 0, big_prev_cb = 0, big_prev_nc = 0;
  // the constant lost-token factors, and a clean candidate bitmap
  load_lost(tb, wpow, sm.fw);
  load_lost(tb, apow, sm.fa);
  for (int w = tid; w < (M + 31) / 32; w += nthr) sm.cbm[w] = 0u;
  {  // exposure counts of the walk, address bit p = token n-1-p
    const int nb = n + tb->k;
    for (int i = tid; i < T * nb; i += nthr) {
      const int sl = i / nb, j = i - sl * nb;
      sm.wc[i] = (uint8_t)(j < n ? tb->cntA[sl][n - 1 - j] : tb->cntD[sl][j - n]);
    }
  }

  QR_TINIT
  const uint32_t seg0 = rp->bucket_base[bkt];
  const uint32_t segn = rp->bucket_base[bkt + 1] - seg0;
  // queue slot of the next trajectory: taken one trajectory ahead, so the
  // atomic's round trip overlaps the current trajectory's work
  uint32_t next_slot = 0;
  if (rp->persistent && tid == 0) next_slot = atomicAdd(&rp->counter[bkt], 1u);
  for (uint32_t iter = 0;; ++iter) {
    if (rp->persistent && tid == 0) sm.misc[0] = (int)next_slot;
    __syncthreads();
    uint32_t qslot;
    if (rp->persistent) {
      qslot = (uint32_t)sm.misc[0];
      if (qslot < segn && tid == 0) next_slot = atomicAdd(&rp->counter[bkt], 1u);
    } else {
      qslot = blockIdx.x + iter * gridDim.x;
    }
    if (qslot >= segn) break;
    const uint32_t tj = rp->order[seg0 + qslot];
    const uint32_t traj = rp->traj0 + tj;
    const uint32_t E = rp->nexpl[tj];
    const uint32_t A = E >> kb;  // explicit addresses
    const uint32_t nct = min(rp->ncand[tj], ccap);
    const uint32_t *__restrict__ cand = rp->cand + (size_t)tj * ccap;
    const uint16_t *__restrict__ xl = pruned ? rp->xlist + (size_t)tj * D : nullptr;
    const uint32_t ref = rp->ref[tj];
    const uint64_t *__restrict__ badg = rp->badbits + (size_t)tj * ((D + 63) >> 6);

    for (uint32_t j = tid; j <= nct; j += nthr) {  // slice boundaries
      const uint32_t cj = j < nct ? cand[j] : 0u;
      const int sj = j < nct ? (int)(cj / (uint32_t)M) + 1 : T;
      const int sp = j > 0 ? (int)(cand[j - 1] / (uint32_t)M) + 1 : 0;
      for (int ss = sp + 1; ss <= sj; ++ss) {
        sm.cstart[ss] = j;
        sm.nxt[ss] = (uint8_t)sj;
      }
      if (pre && j < nct) {  // site, layer and schedule token of every candidate
        const uint32_t q = cj - (uint32_t)(sj - 1) * M;
        const int l = layer_of(q >> 1);
        sm.cdec[j] = q | ((uint32_t)l << 16) | ((uint32_t)tb->tok[sj][l][q & 1u] << 20);
      }
    }
    if (pruned)
      for (int w = tid; w < (D + 31) / 32; w += nthr)
        sm.badl[w] = (uint32_t)(badg[w >> 1] >> (32 * (w & 1)));
    if (tid == 0) {  // work-list rebuild requests: tagged with their slice
      sm.misc[4] = 0;
      sm.misc[5] = 0;
      sm.misc[6] = 0;
    }
    // initial components: data-loading input after the first wall; the sign
    // already holds every fetch phase its live tokens will pick up
    // initial components: data-loading input after the first wall.  Their
    // state words (init_word) are written only at the trajectory's first jump.
    uint64_t alive = 0, devm = 0;  // this thread's live and tier-2 slots (bit j)
    for (uint32_t al = 0; al < apt; ++al) {
      if (tid * apt + al >= A) break;
      alive |= kfull << (al * K2);
    }
    __syncthreads();
    QR_TM(0);

    bool ref_alive = pruned && ref != 0xFFFFFFFFu;
    uint32_t ndev = 0;  // tier-2 components of the block (listed in devl)
    int njumps = 0, first_jump = 0;
    uint32_t jl_n = 0;  // jump-log entries (thread 0, test entry)

    // qubit: rebuild the tier-2 work list, one entry per class of an
    // address's shared lists and one per component with a list of its own
    auto devl_qubit = [&]() {
      uint32_t cnt = 0;
      const int lmax = tb->lmax, kk = tb->k;
      for (uint32_t al = 0; al < apt; ++al) {
        uint64_t cm = 0;
        for (uint64_t m = (devm >> (al * K2)) & kfull; m; m &= m - 1) {
          const uint32_t b = (uint32_t)__ffsll((unsigned long long)m) - 1u;
          if (st[(al * K2 + b) * nthr + tid] & W_SPLIT)
            ++cnt;
          else
            cm |= 1ull << b;
        }
        if (cm) {
          const uint32_t g = tid * apt + al;
          cnt += (uint32_t)__popcll(class_mask(cm, pool[((size_t)g * K2) * rec + 2 + lmax + kk]));
        }
      }
      uint32_t tot;
      uint32_t pos = block_excl_scan_u32(cnt, reinterpret_cast<uint32_t *>(sm.scanb), &tot);
      for (uint32_t al = 0; al < apt; ++al) {
        const uint64_t gm = (devm >> (al * K2)) & kfull;
        if (!gm) continue;
        const uint32_t g = tid * apt + al;
        const uint32_t a = xl ? (uint32_t)xl[g] : g;
        uint64_t cm = 0;
        for (uint64_t m = gm; m; m &= m - 1) {
          const uint32_t b = (uint32_t)__ffsll((unsigned long long)m) - 1u;
          if (st[(al * K2 + b) * nthr + tid] & W_SPLIT)
            devl[pos++] = (g * K2 + b) | (a << 16);
          else
            cm |= 1ull << b;
        }
        if (cm)  // one entry per class of the shared lists
          for (uint64_t mm = class_mask(cm, pool[((size_t)g * K2) * rec + 2 + lmax + kk]); mm; mm &= mm - 1)
            devl[pos++] = (g * K2 + (uint32_t)__ffsll((unsigned long long)mm) - 1u) | (a << 16) | 0x80000000u;
      }
      ndev = tot;
      __syncthreads();
    };

    for (int s = 1; s < T; ++s) {
      if (ndev == 0) {  // without tier-2 components only slices with candidates matter
        s = sm.nxt[s];
        if (s >= T) break;
      }
      if (njumps == 0) {
        // before the first jump the draws follow from the initial labels:
        // go straight to the first slice the block has to evolve
        if (ENC == QUBIT) {
          s = nojump_walk<ENC>(tb, rp, sm, cand, pre, s, traj);
        } else {
          // every wave walks every nw-th slice; the block takes the first stop
          const int nw = nthr >> 6, wv = tid >> 6;
          const int sw = nojump_walk_wave<ENC>(tb, rp, sm, cand, pre, s, traj, wv, nw);
          int *wmin = reinterpret_cast<int *>(sm.scanb);
          if ((tid & 63) == 0) wmin[wv] = sw;
          __syncthreads();
          s = T;
          for (int i = 0; i < nw; ++i) s = min(s, wmin[i]);
          __syncthreads();
        }
        if (s >= T) break;
      }
      const uint32_t cb = sm.cstart[s];
      const int nc = (int)(sm.cstart[s + 1] - cb);
      if (nc == 0 && ndev == 0) continue;
      const bool big = nc > NCS;
      const uint32_t *cd = pre ? sm.cdec + cb : sm.cdec;  // the slice's decoded candidates
      if (nc > 0 && (big || !pre)) {
        if (big) {
          if (big_prev_nc > 0) {
            for (int j = tid; j < big_prev_nc; j += nthr) {
              const uint32_t q = pre ? (sm.cdec[big_prev_cb + j] & 0xFFFFu)
                                     : cand[big_prev_cb + j] - (uint32_t)(big_prev_s - 1) * M;
              sm.cbm[q >> 5] = 0;
            }
            __syncthreads();
          }
          for (int j = tid; j < nc; j += nthr) {
            const uint32_t q = pre ? (sm.cdec[cb + j] & 0xFFFFu) : cand[cb + j] - (uint32_t)(s - 1) * M;
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
      QR_TM(1);

      // tier-2 pass: the listed components (qubit: addresses) follow the
      // gates of slice s literally, spread over all threads of the block
      // (each thread's next entry is fetched one iteration ahead)
      if (ENC == QUBIT && ndev > 0 && tb->store_l[s] >= 0 && !slow_all && sm.misc[6] == s) {
        // before a store: the classes that would store a tagged token into a
        // router split on it (only when a class update or a new list of the
        // previous slice saw such a token: a jump only ever removes tokens).  The address's first class entry does it for
        // all its classes, and only that thread reads or writes the
        // address's split set and records here.  The work list holds an
        // address's class entries together and in ascending class order, and
        // nothing writes it here, so the first entry is found from the list
        // alone: a decision taken from the split set could see it change
        // under another thread's split and split the address twice.
        for (uint32_t i = tid; i < ndev; i += nthr) {
          const uint32_t d = devl[i];
          if (!(d >> 31)) continue;
          const uint32_t cg = d & 0xFFFFu, g = cg >> kb;
          if (i > 0) {
            const uint32_t dp = devl[i - 1];
            if ((dp >> 31) && ((dp & 0xFFFFu) >> kb) == g) continue;
          }
          const uint32_t ow = g / apt, al = g - ow * apt, wbase = al * K2 * nthr + ow;
          uint16_t *r0 = pool + (size_t)g * K2 * rec;
          const uint32_t D = r0[2 + tb->lmax + tb->k];
          uint64_t cm = 0;
          for (int b = 0; b < K2; ++b) {
            const uint32_t w = st[wbase + (uint32_t)b * nthr];
            if ((w & W_ALIVE) && !(w & W_SPLIT)) cm |= 1ull << b;
          }
          const uint64_t cl = class_mask(cm, D);
          if (!cl) continue;
          const uint32_t X = class_store_tokens(tb, s, r0, rec, cl);
          if (X) {
            rec_class_split(r0, rec, tb->k, tb->lmax, cl, D, X, rp->err);
            sm.misc[5] = s;  // the work list is rebuilt before the pass
          }
        }
        __syncthreads();
        if (sm.misc[5] == s) devl_qubit();
      }
      uint32_t dnext = tid < ndev ? devl[tid] : 0u;
      bool t2hit = false;  // a component this thread stepped is hit
      for (uint32_t i = tid; i < ndev; i += nthr) {
        const uint32_t d = dnext;
        if (i + nthr < ndev) dnext = devl[i + nthr];
        const uint32_t c0 = d & 0xFFFFu, a = (d >> 16) & 0x7FFFu;
        uint64_t stepm = 1;  // components c0 + i stepped one by one
        if (ENC == QUBIT && (d >> 31)) {
          // one class of a qubit address's shared lists: the bus words b
          // with b & D = c
          const uint32_t g = c0 >> kb, c = c0 & (uint32_t)(K2 - 1);
          const uint32_t ow = g / apt, al = g - ow * apt;
          const uint32_t wbase = al * K2 * nthr + ow;
          uint16_t *r0 = pool + (size_t)g * K2 * rec;
          const uint32_t D = r0[2 + tb->lmax + tb->k];
          uint64_t mc = 0;  // the class's members
          for (int b = 0; b < K2; ++b) {
            const uint32_t w = st[wbase + (uint32_t)b * nthr];
            if ((w & W_ALIVE) && !(w & W_SPLIT) && ((uint32_t)b & D) == c) mc |= 1ull << b;
          }
          stepm = 0;
          if (mc) {
            uint16_t *recp = r0 + (size_t)c * rec;
            const uint32_t cnt0 = rec_count(recp[0], tb->lmax, rp->err);
            uint32_t cnt = 0, busf = 0, ftok = 0, htok = 0;
            bool fall = false, hall = false, ok = false, split_next = false;
            if (!slow_all && cnt0 + 2 <= 16)  // (a longer shared list splits)
              ok = t2_shared_reg<16>(tb, s, recp, cnt0, a, big, nc, cd, sm.cbm, cnt, busf, fall, ftok, hall, htok,
                                     split_next, rp->err);
            if (ok && split_next) sm.misc[6] = s + 1;  // the next slice runs the pre-split
            if (!ok) {  // one list per member from here on; they take this slice below
              rec_split_class(r0, rec, tb->k, tb->lmax, c, mc, st, wbase, nthr, rp->err);
              stepm = mc;  // (bits: bus words of the address)
              sm.misc[4] = s;  // the work list is rebuilt after the pass
            } else {
              const uint32_t toks = (busf >> 8) & 0xFFu, busm = busf & 0xFFu, intree = toks & ~busm;
              for (uint64_t m = mc; m; m &= m - 1) {
                const uint32_t b = (uint32_t)__ffsll((unsigned long long)m) - 1u;
                const uint32_t widx = wbase + b * nthr;
                const uint32_t w = st[widx];
                const uint32_t live = b & toks;
                const uint32_t e = (w & W_E) + ((w & W_CNT) >> W_CNT_SH);  // exposure through slice s-1
                const uint32_t cb = cnt + (uint32_t)__popc(live & intree);
                const bool flip = fall ^ (bool)(__popc(ftok & live) & 1);
                const bool hit = hall || (htok & live);
                t2hit |= hit;
                // after the last slice a ground component keeps its bus word in the count field
                const uint32_t cf = (s == T - 1 && cb == 0) ? (W_FBUS | ((busm & (~toks | b)) << W_CNT_SH)) : (cb << W_CNT_SH);
                st[widx] = ((w & W_SIGN) ^ (flip ? W_SIGN : 0u)) | (w & (W_ALIVE | W_DEV)) | e | cf | (hit ? W_HIT : 0u);
              }
            }
          }
        }
        const uint32_t cbase = (ENC == QUBIT && (d >> 31)) ? (c0 & ~(uint32_t)(K2 - 1)) : c0;
        for (uint64_t mm = stepm; mm; mm &= mm - 1) {
          const uint32_t c = cbase + (uint32_t)__ffsll((unsigned long long)mm) - 1u;
          const uint32_t g = c >> kb, b = c & (uint32_t)(K2 - 1);
          const uint32_t ow = g / apt, al = g - ow * apt;
          const uint32_t widx = (al * K2 + b) * nthr + ow;
          uint32_t w = st[widx];
          if (!(w & W_ALIVE)) continue;
          const uint32_t cnt0 = (w & W_CNT) >> W_CNT_SH;
          const uint32_t e = (w & W_E) + cnt0;  // exposure through slice s-1
          bool hit;
          uint32_t bus;
          const uint32_t cnt = t2_step<ENC>(tb, s, pool + (size_t)c * rec, cnt0, a, w, slow_all, big, nc,
                                            cd, sm.cbm, hit, bus, rp->err);
          t2hit |= hit;
          // after the last slice a ground list keeps its bus word in the count field
          const uint32_t cf = (s == T - 1 && cnt == 0) ? (W_FBUS | (bus << W_CNT_SH)) : (cnt << W_CNT_SH);
          st[widx] = (w & (W_SIGN | W_ALIVE | W_DEV | W_SPLIT)) | e | cf | (hit ? W_HIT : 0u);
        }
      }
      QR_TM(7);
      if (nc == 0) {  // nothing to draw: only the qubit pass's barrier (and a work-list rebuild)
        if (ENC == QUBIT && ndev > 0) {
          __syncthreads();
          if (sm.misc[4] == s) devl_qubit();  // a class split: spread its components
        }
        continue;
      }
      if (ndev == 0 && !big) {
        // a tier-1 component is excited only where the schedule puts one of
        // its tokens: candidates on token-free sites hit nothing
        bool maybe = false;
        for (int c = 0; c < nc; ++c) maybe |= ((cd[c] >> 20) & 0xFFu) != NONE;
        if (!maybe) continue;
      }

      // owner pass: which of my components does a candidate hit?  The tier-1
      // tests read only this thread's own words and run before the barrier
      // that ends the tier-2 pass; that barrier also collects the hits.
      uint64_t hmask = 0;
      if (njumps == 0) {
        // no jump so far: every component still has its initial label, so
        // the hits follow from the address alone (qubit: bus word b is hit
        // when it shares a live token with a hit data site)
        for (uint32_t al = 0; al < apt; ++al) {
          const uint32_t g = tid * apt + al;
          if (g >= A) break;
          const uint32_t a = xl ? xl[g] : g;
          bool ah;
          uint32_t dh;
          t1_addr_hits<ENC>(tb, s, a, big, nc, cd, sm.cbm, ah, dh);
          uint64_t m;
          if (ENC == QUBIT)
            m = ah ? kfull : (kfull & ~subsets_of(~dh & kmask, tb->k));
          else
            m = (ah || (mem[a] & kmask & tb->dmask[s] & dh)) ? 1ull : 0ull;
          hmask |= m << (al * K2);
        }
      } else {
        int cur = -1;
        uint32_t memw = 0, dh = 0;
        bool ah = false;
        for (uint64_t m = alive & ~devm; m; m &= m - 1) {  // tier 1
          const int j = __ffsll((unsigned long long)m) - 1;
          const int al = j >> kb;
          if (al != cur) {
            cur = al;
            const uint32_t g = tid * apt + (uint32_t)al;
            const uint32_t a = xl ? xl[g] : g;
            memw = ENC == QUTRIT ? mem[a] : 0u;
            t1_addr_hits<ENC>(tb, s, a, big, nc, cd, sm.cbm, ah, dh);
          }
          const uint32_t w = st[j * nthr + tid];
          const uint32_t live = (w >> W_LIVE_SH) & 0xFFu;
          const uint32_t df = ENC == QUBIT ? live : (live & memw & tb->dmask[s]);
          if (ah || (df & dh)) hmask |= 1ull << j;
        }
      }
      const bool any_hit = __syncthreads_or(hmask != 0ull || t2hit);
      if (ENC == QUBIT && ndev > 0 && sm.misc[4] == s) devl_qubit();  // a class split in the pass
      for (uint64_t m = devm; m; m &= m - 1) {  // tier 2: hit flags from the tier-2 pass
        const int j = __ffsll((unsigned long long)m) - 1;
        if (st[j * nthr + tid] & W_HIT) hmask |= 1ull << j;
      }
      QR_TM(2);
      if (!any_hit) continue;  // J is empty

      // a draw slice: weights of every component before this slice's layer
      load_factors<ENC>(tb, s - 1, tb->ftab_w, sm.fw, sm.fmisc);
      __syncthreads();
      const double wr = sm.fmisc[0];
      double acc[3] = {0.0, 0.0, 0.0};  // w_empty, w_hit, good branches
      if (njumps == 0) {
        // initial labels: live tokens = bus word (qubit), every bit (qutrit).
        // Only the hit components are summed; every address, explicit or
        // good, is still on its no-jump orbit, so the total weight is the
        // slice's closed-form sum over all addresses.
        for (uint32_t al = 0; al < apt; ++al) {
          const uint64_t hm = (hmask >> (al * K2)) & kfull;
          if (!hm) continue;
          const uint32_t g = tid * apt + al;
          const uint32_t a = xl ? xl[g] : g;
          const double wa = fA(sm.fw, a) * wr;
          for (uint64_t m = hm; m; m &= m - 1) {
            const uint32_t b = (uint32_t)__ffsll((unsigned long long)m) - 1u;
            acc[1] += wa * sm.fw[F_D + (ENC == QUBIT ? b : (kmask & mem[a]))];
          }
        }
      } else {
        int cur = -1;
        uint32_t memw = 0;
        double wa = 0.0;
        for (uint64_t m = alive; m; m &= m - 1) {
          const int j = __ffsll((unsigned long long)m) - 1;
          const uint32_t w = st[j * nthr + tid];
          double wt;
          if (w & W_DEV) {
            wt = wpow[w & W_E];
          } else {
            const int al = j >> kb;
            if (al != cur) {
              cur = al;
              const uint32_t g = tid * apt + (uint32_t)al;
              const uint32_t a = xl ? xl[g] : g;
              memw = ENC == QUTRIT ? mem[a] : 0u;
              wa = fA(sm.fw, a) * wr;
            }
            const uint32_t live = (w >> W_LIVE_SH) & 0xFFu;
            const uint32_t dv = ENC == QUBIT ? live : (live & memw);
            wt = wa * sm.fw[F_D + dv] * sm.fw[F_K + (w & W_EK)];
          }
          if ((hmask >> j) & 1ull)
            acc[1] += wt;
          else
            acc[0] += wt;
        }
      }
      const double my_hit_w = acc[1];
      if (ref_alive && njumps > 0) {
        // good branches other than the reference, on their no-jump orbits
        for (int i = tid; i < D; i += nthr) {
          if ((uint32_t)i == ref || ((sm.badl[i >> 5] >> (i & 31)) & 1u)) continue;
          double x = fA(sm.fw, (uint32_t)i);
          if (ENC == QUTRIT) x *= sm.fw[F_D + (mem[i] & kmask)];
          acc[2] += x;
        }
      }
      double *rbuf = sm.red + (s & 1) * (nthr >> 6) * 8;
      block_sum<3>(acc, rbuf);
      QR_TM(3);
      double sd = wr;  // qutrit: the router factor; qubit: the bus-word sum
      if (ENC == QUBIT) {
        sd = 0.0;
        for (int b = 0; b < K2; ++b) sd += sm.fw[F_D + b];
      }
      const double wgood = ref_alive ? acc[2] * sd : 0.0;
      const double u = rp->forced ? rp->uaux[s] : uniform53(rp->seed, (uint32_t)s, 0, traj, 2u);
      const double wall = njumps == 0 ? tb->ctot[s - 1] : acc[0] + wgood + acc[1];
      const double w0 = njumps == 0 ? wall - acc[1] : acc[0] + wgood;
      const double r = u * wall;
      if (r < w0) continue;  // J empty: K0 already accounted
      const double r2 = r - w0;

      // auxiliary component x*: the empty-mask block first, then the other
      // components in slot order (initial-label order)
      if (tid == 0) {  // (published by the scan's barrier)
        sm.misc[1] = -1;
        sm.misc[2] = 0;
      }
      const double excl = block_excl_scan(my_hit_w, sm.scanb);
      if (my_hit_w > 0.0 && excl <= r2) atomicMax(&sm.misc[1], tid);
      __syncthreads();
      if (sm.misc[1] == tid) {
        double cum = excl;
        int pick = -1, last = -1;
        for (uint32_t al = 0; al < apt && pick < 0; ++al) {
          const uint32_t g = tid * apt + al;
          if (g >= A) break;
          const uint32_t a = xl ? xl[g] : g;
          const uint32_t memw = ENC == QUTRIT ? mem[a] : 0u;
          for (int b = 0; b < K2; ++b) {
            const uint32_t j = al * K2 + b;
            if (!((hmask >> j) & 1ull)) continue;
            const uint32_t w = njumps == 0 ? init_word<ENC>(mem[a], (uint32_t)b, kmask) : st[j * nthr + tid];
            double wt;
            if (!(w & W_DEV)) {
              const uint32_t live = (w >> W_LIVE_SH) & 0xFFu;
              const uint32_t dv = ENC == QUBIT ? live : (live & memw);
              wt = fA(sm.fw, a) * wr * sm.fw[F_D + dv] * sm.fw[F_K + (w & W_EK)];
            } else {
              wt = wpow[w & W_E];
            }
            last = (int)j;
            cum += wt;
            if (cum > r2) {
              pick = (int)j;
              break;
            }
          }
        }
        if (pick < 0) pick = last;
        // J = the slice's candidates among x*'s excited sites, with levels
        int nJ = 0;
        const uint32_t al = (uint32_t)pick / K2, b = (uint32_t)pick % K2;
        const uint32_t g = tid * apt + al;
        const uint32_t a = xl ? xl[g] : g;
        const uint32_t memw = ENC == QUTRIT ? mem[a] : 0u;
        const uint32_t w = njumps == 0 ? init_word<ENC>(mem[a], b, kmask) : st[pick * nthr + tid];
        if (!(w & W_DEV)) {
          const uint32_t live = (w >> W_LIVE_SH) & 0xFFu;
          if (!big) {
            for (int c = 0; c < nc; ++c) {
              const uint32_t q = cd[c] & 0xFFFFu;
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
        } else if (ENC == QUBIT && !(w & W_SPLIT)) {
          // a shared list (x*'s class): its address entries and the tokens x* carries
          const uint16_t *r0 = pool + (size_t)g * K2 * rec;
          const uint16_t *rs = r0 + (size_t)(b & r0[2 + tb->lmax + tb->k]) * rec;
          const uint32_t live = b & ((uint32_t)rs[1] >> 8);
          const uint32_t nrs = rec_count(rs[0], tb->lmax, rp->err);
          for (uint32_t c = 0; c < nrs; ++c) {
            const uint32_t q = rs[2 + c];
            if ((big ? cand_bm(sm.cbm, q) : cand_list(cd, nc, q)) && nJ < JMAX) sm.Jb[nJ++] = q | (1u << 16);
          }
          for (int t = 0; t < tb->k; ++t) {
            const uint32_t q = rs[2 + tb->lmax + t];
            if (!((live >> t) & 1u) || q == EMPTY) continue;
            if ((big ? cand_bm(sm.cbm, q) : cand_list(cd, nc, q)) && nJ < JMAX) sm.Jb[nJ++] = q | (1u << 16);
          }
        } else {
          Rec<ENC> R{pool + (size_t)(g * K2 + b) * rec};
          R.bound(tb->lmax, rp->err);
          for (int c = 0; c < R.cnt(); ++c) {
            const uint32_t x = R.raw(c), q = x & Rec<ENC>::SM;
            const bool isc = big ? cand_bm(sm.cbm, q) : cand_list(cd, nc, q);
            if (!isc) continue;
            const uint32_t lev = (ENC == QUTRIT && (x & LV_R_BIT)) ? 2u : 1u;
            if (nJ < JMAX) sm.Jb[nJ++] = q | (lev << 16);
          }
        }
        sm.misc[2] = nJ;
      }
      __syncthreads();
      const int nJ = sm.misc[2];
      QR_TM(4);
      if (nJ == 0) continue;
      if (rp->jlog && tid == 0) {
        for (int c = 0; c < nJ; ++c, ++jl_n)
          if (jl_n < rp->jcap) rp->jlog[(size_t)tj * rp->jcap + jl_n] = sm.Jb[c] | ((uint32_t)s << 24);
      }

      // K_J on every component: survivors carry every site of J
      uint32_t mydev = 0;
      for (uint32_t al = 0; al < apt; ++al) {
        const uint32_t g = tid * apt + al;
        if (g >= A) break;
        const uint32_t a = xl ? xl[g] : g;
        const uint32_t memw = ENC == QUTRIT ? mem[a] : 0u;
        uint64_t skip = 0;  // components already handled with their shared list
        if (ENC == QUBIT) {
          const uint32_t base = al * K2;
          const uint64_t am = (alive >> base) & kfull;
          if (!am) continue;
          const bool t2 = ((devm >> base) & kfull) != 0ull;
          if (t2) {
            // the members on shared lists, class by class: J's sites must be
            // on the class's list, J's tagged tokens carried
            uint16_t *r0 = pool + (size_t)g * K2 * rec;
            const int kk = tb->k, lmax = tb->lmax;
            const uint32_t D = r0[2 + lmax + kk];
            uint64_t cm = 0;
            for (uint64_t m = am; m; m &= m - 1) {
              const uint32_t b = (uint32_t)__ffsll((unsigned long long)m) - 1u;
              if (!(st[(base + b) * nthr + tid] & W_SPLIT)) cm |= 1ull << b;
            }
            for (uint64_t mm = class_mask(cm, D); mm; mm &= mm - 1) {
              const uint32_t c = (uint32_t)__ffsll((unsigned long long)mm) - 1u;
              uint16_t *rs = r0 + (size_t)c * rec;
              Rec<ENC> R{rs};
              R.bound(lmax, rp->err);
              const uint32_t busf = rs[1], toks = (busf >> 8) & 0xFFu;
              bool okA = true;
              uint32_t need = 0;
              for (int cc = 0; cc < nJ && okA; ++cc) {
                const uint32_t q = sm.Jb[cc] & 0xFFFFu;
                if (R.find_site(q) >= 0) continue;
                int tq = -1;
                for (int t = 0; t < kk; ++t)
                  if (((toks >> t) & 1u) && rs[2 + lmax + t] == q) tq = t;
                if (tq < 0)
                  okA = false;
                else
                  need |= 1u << tq;
              }
              uint64_t mc = 0, surv = 0;
              for (uint64_t m = cm; m; m &= m - 1) {
                const uint32_t b = (uint32_t)__ffsll((unsigned long long)m) - 1u;
                if ((b & D) != c) continue;
                mc |= 1ull << b;
                if (okA && !(need & ~(b & toks))) surv |= 1ull << b;
              }
              if (surv) {
                for (int cc = 0; cc < nJ; ++cc) {
                  const int jj = R.find_site(sm.Jb[cc] & 0xFFFFu);
                  if (jj >= 0) R.remove(jj);
                }
                for (int t = 0; t < kk; ++t)
                  if ((need >> t) & 1u) rs[2 + lmax + t] = (uint16_t)EMPTY;
                rs[1] = (uint16_t)(busf & ~(need << 8));
              }
              const uint32_t toks2 = toks & ~need, busm = busf & 0xFFu;
              for (uint64_t m = mc; m; m &= m - 1) {
                const uint32_t b = (uint32_t)__ffsll((unsigned long long)m) - 1u;
                const uint32_t j = base + b;
                if (!((surv >> b) & 1ull)) {
                  st[j * nthr + tid] = 0u;
                  alive &= ~(1ull << j);
                  devm &= ~(1ull << j);
                  continue;
                }
                const uint32_t w = st[j * nthr + tid];
                const uint32_t cnt = ((w & W_CNT) >> W_CNT_SH) - (uint32_t)nJ;
                const uint32_t cf = (s == T - 1 && cnt == 0) ? (W_FBUS | ((busm & (~toks2 | b)) << W_CNT_SH)) : (cnt << W_CNT_SH);
                st[j * nthr + tid] = (w & (W_SIGN | W_ALIVE | W_DEV | W_E)) | cf;
              }
            }
            skip = cm;
            if (!(am & ~cm)) continue;  // (members with lists of their own: below)
          }
          if (!t2) {
            // tier 1: J's data tokens, and whether J holds an address token
            // (then the survivors turn tier 2): the same for every bus word
            bool devJ = false;
            uint32_t kill = 0;
            for (int c = 0; c < nJ; ++c) {
              const uint32_t q = sm.Jb[c] & 0xFFFFu;
              const uint32_t tk = tb->tok[s][layer_of(q >> 1)][q & 1u];
              if (tk < (uint32_t)n || tk == NONE)
                devJ = true;
              else
                kill |= 1u << (tk - (uint32_t)n);
            }
            if (devJ) {
              uint64_t surv = 0;
              uint32_t toks = 0;  // data tokens the survivors still carry
              for (uint64_t m = am; m; m &= m - 1) {
                const uint32_t b = (uint32_t)__ffsll((unsigned long long)m) - 1u;
                const uint32_t w = njumps == 0 ? init_word<ENC>(mem[a], b, kmask) : st[(base + b) * nthr + tid];
                const uint32_t live = (w >> W_LIVE_SH) & 0xFFu;
                bool ok = true;
                for (int c = 0; c < nJ && ok; ++c) {
                  const uint32_t x = sm.Jb[c];
                  ok = t1_level<ENC>(tb, s, a, live, 0u, x & 0xFFFFu) == (int)(x >> 16);
                }
                if (ok) {
                  surv |= 1ull << b;
                  toks |= live & ~kill;
                }
              }
              uint32_t caddr = 0, busm = 0;
              if (surv) {
                // the address's shared list: every excited site but J's
                // (lost), written once
                uint16_t *rs = pool + (size_t)g * K2 * rec;
                bool ovf = false;
                int qs[MAXN];  // the address tokens' sites, loaded together
#pragma unroll
                for (int t = 0; t < MAXN; ++t) qs[t] = t < n ? t1_site(tb, s, a, t) : -1;
#pragma unroll
                for (int t = 0; t < MAXN; ++t) {
                  const int q = qs[t];
                  if (q < 0 || !((a >> (n - 1 - t)) & 1u)) continue;
                  bool inJ = false;
                  for (int c = 0; c < nJ; ++c) inJ |= (sm.Jb[c] & 0xFFFFu) == (uint32_t)q;
                  if (inJ) continue;
                  if (caddr < (uint32_t)tb->lmax)
                    rs[2 + caddr++] = (uint16_t)q;
                  else
                    ovf = true;
                }
                const int nsl = s + 1 < T ? tb->store_l[s + 1] : -1;
                for (int bb = 0; bb < tb->k; ++bb) {
                  const int q = ((toks >> bb) & 1u) ? t1_site(tb, s, a, n + bb) : -1;
                  if (((toks >> bb) & 1u) && q < 0) busm |= 1u << bb;  // not yet in, or already back on the bus
                  rs[2 + tb->lmax + bb] = (uint16_t)(q >= 0 ? (uint32_t)q : EMPTY);
                  if (q >= 0 && nsl >= 0 && layer_of((uint32_t)q >> 1) == nsl) sm.misc[6] = s + 1;
                }
                if (ovf) atomicOr(rp->err, ERR_LIST);
                rs[0] = (uint16_t)caddr;
                rs[1] = (uint16_t)(busm | (toks << 8));
                rs[2 + tb->lmax + tb->k] = 0;  // one class
              }
              const uint32_t intree = toks & ~busm;
              uint32_t future = 0;  // fetch phases still ahead, picked up literally in tier 2
              for (int bb = 0; bb < tb->k; ++bb)
                if (3 * n + 2 * bb + 1 > s) future |= 1u << bb;
              for (uint64_t m = am; m; m &= m - 1) {
                const uint32_t b = (uint32_t)__ffsll((unsigned long long)m) - 1u;
                const uint32_t j = base + b;
                if (!((surv >> b) & 1ull)) {
                  st[j * nthr + tid] = 0u;
                  alive &= ~(1ull << j);
                  devm &= ~(1ull << j);
                  continue;
                }
                const uint32_t w = njumps == 0 ? init_word<ENC>(mem[a], b, kmask) : st[j * nthr + tid];
                const uint32_t live = (w >> W_LIVE_SH) & 0xFFu;
                // exposure through slice s (J's sites excluded)
                const uint32_t e = t1_exposure<ENC>(tb, sm.wc + s * (n + tb->k), s, a, live, w & W_EK) - (uint32_t)nJ;
                uint32_t sign = w & W_SIGN;
                if (__popc(live & mem[a] & future) & 1) sign ^= W_SIGN;
                const uint32_t cb = caddr + (uint32_t)__popc(b & toks & intree);
                const uint32_t cf = (s == T - 1 && cb == 0) ? (W_FBUS | ((b & toks & busm) << W_CNT_SH)) : (cb << W_CNT_SH);
                st[j * nthr + tid] = (W_ALIVE | W_DEV | sign) | (e - cb) | cf;
                devm |= 1ull << j;
              }
              continue;
            }
          }
          // components with lists of their own, or no address token in J:
          // one component at a time
        }
        for (int b = 0; b < K2; ++b) {
          if ((skip >> b) & 1ull) continue;
          const uint32_t j = al * K2 + b;
          uint32_t w = njumps == 0 ? init_word<ENC>(mem[a], (uint32_t)b, kmask) : st[j * nthr + tid];
          if (!(w & W_ALIVE)) continue;
          uint16_t *recp = pool + (size_t)(g * K2 + b) * rec;
          if (!(w & W_DEV)) {
            uint32_t live = (w >> W_LIVE_SH) & 0xFFu;
            bool ok = true, dev = false;
            for (int c = 0; c < nJ && ok; ++c) {
              const uint32_t x = sm.Jb[c], q = x & 0xFFFFu;
              ok = t1_level<ENC>(tb, s, a, live, memw, q) == (int)(x >> 16);
            }
            if (!ok) {
              st[j * nthr + tid] = 0u;
              alive &= ~(1ull << j);
              devm &= ~(1ull << j);
              continue;
            }
            uint32_t kill = 0;
            for (int c = 0; c < nJ; ++c) {
              const uint32_t q = sm.Jb[c] & 0xFFFFu;
              const uint32_t tk = tb->tok[s][layer_of(q >> 1)][q & 1u];
              if (tk < (uint32_t)n)
                dev = true;
              else
                kill |= 1u << (tk - (uint32_t)n);
            }
            if (dev) {
              // exposure through slice s and the phases fetched so far
              const uint32_t dv = ENC == QUBIT ? live : (live & memw);
              const uint32_t e = t1_exposure<ENC>(tb, sm.wc + s * (n + tb->k), s, a, dv, w & W_EK) - (uint32_t)nJ;
              uint32_t sign = w & W_SIGN;
              if (ENC == QUBIT) {
                uint32_t future = 0;
                for (int bb = 0; bb < tb->k; ++bb)
                  if (3 * n + 2 * bb + 1 > s) future |= 1u << bb;
                if (__popc(live & mem[a] & future) & 1) sign ^= W_SIGN;
              }
              // the record: every excited site but J's (lost), written once
              uint32_t cnt = 0, bus = 0;
              bool ovf = false;
              auto put = [&](uint32_t raw) {
                for (int c = 0; c < nJ; ++c) {
                  const uint32_t xj = sm.Jb[c], qj = xj & 0xFFFFu;
                  if (raw == ((ENC == QUTRIT && (xj >> 16) == 2u) ? (qj | LV_R_BIT) : qj)) return;
                }
                if (cnt < (uint32_t)tb->lmax)
                  recp[2 + cnt++] = (uint16_t)raw;
                else
                  ovf = true;
              };
              int qs[MAXN];  // the tokens' sites, loaded together
#pragma unroll
              for (int t = 0; t < MAXN; ++t) qs[t] = t < n ? t1_site(tb, s, a, t) : -1;
#pragma unroll
              for (int t = 0; t < MAXN; ++t) {
                const int q = qs[t];
                if (q < 0) continue;
                const bool abit = (a >> (n - 1 - t)) & 1u;
                if (ENC == QUTRIT && (q & 1) == 0)
                  put((uint32_t)q | (abit ? LV_R_BIT : 0u));
                else if (abit)
                  put((uint32_t)q);
              }
              for (int bb = 0; bb < tb->k; ++bb) {
                const int q = t1_site(tb, s, a, n + bb);
                if (ENC == QUBIT) {
                  const bool lb = (live >> bb) & 1u;
                  if (q >= 0) {
                    if (lb) put((uint32_t)q);
                  } else if (lb) {
                    bus |= 1u << bb;  // not yet in, or already back on the bus
                  }
                } else {
                  const bool vb = ((memw & live) >> bb) & 1u;
                  if (q >= 0) {
                    if (((tb->dmask[s] >> bb) & 1u) && vb) put((uint32_t)q);
                  } else if (s >= 4 * n + 2 * bb + 1 && vb) {
                    bus |= 1u << bb;  // fetched value already on the bus
                  }
                }
              }
              if (ovf) atomicOr(rp->err, ERR_LIST);
              recp[0] = (uint16_t)cnt;
              recp[1] = (uint16_t)bus;
              // after the last slice a ground list keeps its bus word in the count field
              const uint32_t cf = (s == T - 1 && cnt == 0) ? (W_FBUS | (bus << W_CNT_SH)) : (cnt << W_CNT_SH);
              w = (W_ALIVE | W_DEV | sign) | (e - cnt) | cf;
            } else {
              uint32_t ek = w & W_EK;
              uint32_t sign = w & W_SIGN;
              for (int bb = 0; bb < tb->k; ++bb) {
                if (!((kill >> bb) & 1u)) continue;
                ek += tb->cntD[s - 1][bb];
                // a token lost before its fetch never picks up the phase
                if (ENC == QUBIT && s < 3 * n + 2 * bb + 1 && ((mem[a] >> bb) & 1u)) sign ^= W_SIGN;
              }
              live &= ~kill;
              w = W_ALIVE | sign | (live << W_LIVE_SH) | ek;
            }
          } else {
            Rec<ENC> R{recp};
            R.bound(tb->lmax, rp->err);
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
              alive &= ~(1ull << j);
              devm &= ~(1ull << j);
              continue;
            }
            const uint32_t cnt = ((w & W_CNT) >> W_CNT_SH) - (uint32_t)nJ;
            const uint32_t cf = (s == T - 1 && cnt == 0) ? (W_FBUS | ((uint32_t)R.r[1] << W_CNT_SH)) : (cnt << W_CNT_SH);
            w = (w & (W_SIGN | W_ALIVE | W_DEV | W_SPLIT | W_E)) | cf;
          }
          st[j * nthr + tid] = w;
          if (w & W_DEV) {
            ++mydev;
            devm |= 1ull << j;
          }
        }
      }
      ref_alive = false;  // a good branch never carries a candidate site
      ++njumps;
      if (!first_jump) first_jump = s;
      // rebuild the tier-2 work list in slot order
      if (ENC == QUBIT) {
        devl_qubit();
      } else {
        uint32_t tot;
        uint32_t pos = block_excl_scan_u32(mydev, reinterpret_cast<uint32_t *>(sm.scanb), &tot);
        int cur = -1;
        uint32_t a = 0;
        for (uint64_t m = devm; m; m &= m - 1) {
          const uint32_t j = (uint32_t)__ffsll((unsigned long long)m) - 1u;
          const uint32_t g = tid * apt + (j >> kb);
          if ((int)(j >> kb) != cur) {
            cur = (int)(j >> kb);
            a = xl ? xl[g] : g;
          }
          devl[pos++] = (g * K2 + (j & (uint32_t)(K2 - 1))) | (a << 16);
        }
        ndev = tot;
        __syncthreads();
      }
      QR_TM(5);
    }

    if (big_prev_nc > 0) {  // leave the candidate bitmap clean
      __syncthreads();
      for (int j = tid; j < big_prev_nc; j += nthr) {
        const uint32_t q = pre ? (sm.cdec[big_prev_cb + j] & 0xFFFFu)
                               : cand[big_prev_cb + j] - (uint32_t)(big_prev_s - 1) * M;
        sm.cbm[q >> 5] = 0;
      }
      big_prev_nc = 0;
    }

    // second wall, tree measurement and fidelity (Alg. 1 steps 4-6)
    __syncthreads();
    if (rp->jn && tid == 0) rp->jn[tj] = jl_n;
    if (njumps == 0) {
      if (rp->exp && tj == 0) {  // every branch on its no-jump orbit
        for (uint32_t x = tid; x < (uint32_t)(D * K2); x += nthr) {
          const uint32_t a = x / (uint32_t)K2, b = x % (uint32_t)K2;
          const uint32_t w = init_word<ENC>(mem[a], b, kmask);
          const uint32_t dv = ENC == QUBIT ? b : (mem[a] & kmask);
          export_ground<ENC>(tb, rp->exp, a, b, dv, (w & W_SIGN) != 0, t1_final_exposure<ENC>(tb, a, dv, 0u));
        }
      }
      // no jump: every branch ends on its no-jump orbit in the ground
      // configuration, so the sums are the context's closed-form constants
      if (tid == 0) {
        const double ov = tb->ov_nojump, wt = tb->w_nojump;
        const double norm = 1.0 / ((double)D * (double)K2);
        const double uf = rp->forced ? rp->ufin : uniform53(rp->seed, 0, 0, traj, 3u);
        const bool qg = uf * wt < wt;
        rp->fid[tj] = (qg && wt > 0.0) ? ov * ov / wt * norm : 0.0;
        if (rp->st) {
          qram_traj_stats o;
          o.n_cand = rp->ncand[tj];
          o.n_bad = rp->nbad[tj];
          o.ref_addr = ref;
          o.n_explicit = E;
          o.n_jumps = 0;
          o.first_jump_slice = 0;
          o.ref_survived = (uint8_t)(ref != 0xFFFFFFFFu);
          o.q_ground = (uint8_t)qg;
          o.flags = (uint8_t)((rp->ncand[tj] > ccap ? 1 : 0));
          o.pad = 0;
          o.fid_pre = wt > 0.0 ? ov * ov / wt * norm : 0.0;
          rp->st[tj] = o;
        }
      }
      QR_TM(6);
      continue;
    }
    load_factors<ENC>(tb, T - 1, tb->ftab_w, sm.fw, sm.fmisc);
    load_factors<ENC>(tb, T - 1, tb->ftab_a, sm.fa, sm.fmisc + 1);
    __syncthreads();
    const double wr = sm.fmisc[0], ar = sm.fmisc[1];
    double fin[5] = {0, 0, 0, 0, 0};  // overlap, w_ground, w_total, good a-sum, good w-sum
    {
      int cur = -1;
      uint32_t memw = 0, g = 0;
      double wa = 0.0, aa = 0.0;
      uint32_t acur = 0;
      for (uint64_t m = alive; m; m &= m - 1) {
        const int j = __ffsll((unsigned long long)m) - 1;
        const int al = j >> kb, b = j & (K2 - 1);
        if (al != cur) {
          cur = al;
          g = tid * apt + (uint32_t)al;
          const uint32_t a = xl ? xl[g] : g;
          acur = a;
          memw = mem[a] & kmask;
          wa = fA(sm.fw, a) * wr;
          aa = fA(sm.fa, a) * ar;
        }
        const uint32_t w = st[j * nthr + tid];
        if (rp->exp && tj == 0) export_explicit<ENC>(tb, rp->exp, pool, rec, g, acur, (uint32_t)b, w, memw);
        double wt, at;
        bool ground;
        uint32_t bus;
        if (!(w & W_DEV)) {
          const uint32_t live = (w >> W_LIVE_SH) & 0xFFu;
          const uint32_t dv = ENC == QUBIT ? live : (live & memw);
          wt = wa * sm.fw[F_D + dv] * sm.fw[F_K + (w & W_EK)];
          at = aa * sm.fa[F_D + dv] * sm.fa[F_K + (w & W_EK)];
          ground = true;
          bus = dv;
        } else {
          const bool fb = (w & W_FBUS) != 0u;
          const uint32_t cnt = fb ? 0u : (w & W_CNT) >> W_CNT_SH;
          const uint32_t e = (w & W_E) + cnt;
          wt = wpow[e];
          at = apow[e];
          ground = cnt == 0;
          if (fb) {
            bus = (w & W_CNT) >> W_CNT_SH;
          } else if (!ground) {
            bus = 0u;
          } else if (ENC == QUBIT && !(w & W_SPLIT)) {
            const uint16_t *r0 = pool + (size_t)g * K2 * rec;
            const uint32_t bf = r0[(size_t)(b & r0[2 + tb->lmax + tb->k]) * rec + 1];
            bus = bf & (~(bf >> 8) | (uint32_t)b) & 0xFFu;
          } else {
            bus = pool[(size_t)(g * K2 + b) * rec + 1];
          }
        }
        fin[2] += wt;
        if (!ground) continue;
        fin[1] += wt;
        if (ENC == QUBIT) {
          const bool neg = ((w & W_SIGN) != 0) ^ (bool)(__popc(bus & memw) & 1);
          fin[0] += neg ? -at : at;
        } else if (bus == memw) {
          fin[0] += at;
        }
      }
    }
    if (ref_alive) {
      for (int i = tid; i < D; i += nthr) {
        if ((uint32_t)i == ref || ((sm.badl[i >> 5] >> (i & 31)) & 1u)) continue;
        double xa = fA(sm.fa, (uint32_t)i), xw = fA(sm.fw, (uint32_t)i);
        if (ENC == QUTRIT) {
          xa *= sm.fa[F_D + (mem[i] & kmask)];
          xw *= sm.fw[F_D + (mem[i] & kmask)];
        }
        fin[3] += xa;
        fin[4] += xw;
      }
    }
    block_sum<5>(fin, sm.red);
    if (tid == 0) {
      double ov = fin[0], wg = fin[1], wt = fin[2];
      if (ref_alive) {  // the predicted good groups (Theorem 3 / Proposition 1)
        double sa = ar, sw = wr;
        if (ENC == QUBIT) {
          sa = sw = 0.0;
          for (int b = 0; b < K2; ++b) {
            sw += sm.fw[F_D + b];
            sa += sm.fa[F_D + b];
          }
        }
        ov += fin[3] * sa;
        wg += fin[4] * sw;
        wt += fin[4] * sw;
      }
      const double uf = rp->forced ? rp->ufin : uniform53(rp->seed, 0, 0, traj, 3u);
      const bool qg = uf * wt < wg;
      const double norm = 1.0 / ((double)D * (double)K2);
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
    QR_TM(6);
  }
  QR_TFLUSH
}

}  // namespace

uint32_t evolve_lds_bytes(int M, int D, int threads, uint32_t cdec_cap,
                          uint32_t e_cap, bool state_lds, uint32_t walk_bytes) {
  return fixed_bytes(M, D, threads, cdec_cap, walk_bytes) + (state_lds ? e_cap * 4u : 0u);
}

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

#ifdef QR_PHASE_TIMERS
extern "C" int qram_probe_phase_cycles(unsigned long long *out, int reset) {
  hipError_t e = hipMemcpyFromSymbol(out, HIP_SYMBOL(qr_phase_cycles), sizeof(unsigned long long) * 16);
  if (reset) {
    unsigned long long z[16] = {};
    e = hipMemcpyToSymbol(HIP_SYMBOL(qr_phase_cycles), z, sizeof(z));
  }
  return (int)e;
}
#endif

hipError_t evolve_prepare(int lds_max, int *dyn_max) {
  hipError_t e = hipSuccess;
  const void *fns[4] = {reinterpret_cast<const void *>(&k_evolve<QUBIT, true>),
                        reinterpret_cast<const void *>(&k_evolve<QUBIT, false>),
                        reinterpret_cast<const void *>(&k_evolve<QUTRIT, true>),
                        reinterpret_cast<const void *>(&k_evolve<QUTRIT, false>)};
  int dyn = lds_max;
  for (const void *f : fns) {  // the compiler's own shared memory comes first
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, f) == hipSuccess) dyn = std::min(dyn, lds_max - (int)fa.sharedSizeBytes);
  }
  for (const void *f : fns) {
    const hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, dyn);
    if (r != hipSuccess) e = r;
  }
  *dyn_max = dyn;
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
