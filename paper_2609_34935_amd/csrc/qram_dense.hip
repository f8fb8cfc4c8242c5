// Dense whole-register evolution of the loading circuit for tiny trees: the
// cross-check of App. C on the GPU.  The register holds every digit of the
// machine (address bits, bus bits, every tree site) as an ordinary basis
// label, with no branch bookkeeping and no sampling:
//   - a density matrix under the explicit channels of every slice (n <= 2):
//     the gates, depolarizing on App. C's active positions, amplitude
//     damping on every tree site (Eq. kraus / kraus-tri), and two further
//     channels the outlook of Sec. VII names as candidates, dephasing and
//     heating (both with a diagonal no-jump operator);
//   - a state vector under a given history of joint damping outcomes and
//     depolarizing faults (n <= 3), to compare component by component with
//     the branch simulators.
// Digits, most significant first: address bit t (t = 0 is the root's bit),
// bus bit b, tree site q (router 2v, data slot 2v+1); a qutrit router has
// three levels (W, L, R = 0, 1, 2), every other digit two.  The time-slice
// schedule is the context's own (App. C reads it from the same scheduler).

#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "qram_device.h"
#include "qram_internal.h"

namespace qr {
namespace {

struct DDims {
  int n, k, M, nd, enc;
  uint64_t N;
  uint64_t pv[DENSE_MAXD];  // place values, last digit fastest
  int rad[DENSE_MAXD];
};

__device__ __forceinline__ void dec(const DDims &d, uint64_t x, int *g) {
  for (int i = 0; i < d.nd; ++i) g[i] = (int)((x / d.pv[i]) % (uint64_t)d.rad[i]);
}

__device__ __forceinline__ uint64_t enc_idx(const DDims &d, const int *g) {
  uint64_t x = 0;
  for (int i = 0; i < d.nd; ++i) x += (uint64_t)g[i] * d.pv[i];
  return x;
}

__device__ __forceinline__ void swp(int &a, int &b) {
  const int t = a;
  a = b;
  b = t;
}

// The gates of slice s on one basis label (digits g); returns the sign the
// qubit fetch puts on it.  Events of one slice act on disjoint digits, so
// their order does not matter.
__device__ double slice_gates(const Tables *__restrict__ tb, const DDims &d, int s, int *g) {
  const int n = d.n, k = d.k;
  int *A = g, *B = g + n, *S = g + n + k;
  double ph = 1.0;
  const int bb = tb->bus_b[s];
  if (bb >= 0) swp(B[bb], S[1]);  // SWAP(bus_b, d_0)
  const int ct = tb->copy_t[s];
  if (ct >= 0) S[1] ^= A[ct];  // CNOT of address bit t into d_0
  const uint32_t cm = tb->cswap[s];
  for (int l = 0; l + 1 < n; ++l) {
    if (!((cm >> l) & 1u)) continue;
    for (int v = (1 << l) - 1; v < (2 << l) - 1; ++v) {
      const int r = S[2 * v];
      int child;
      if (d.enc == QUBIT)
        child = 2 * v + 1 + r;
      else if (r == 0)
        continue;  // W blocks the swap
      else
        child = 2 * v + (r == 1 ? 1 : 2);
      swp(S[2 * v + 1], S[2 * child + 1]);
    }
  }
  const int fb = tb->fetch_b[s];
  if (fb >= 0) {
    const int v0 = (1 << (n - 1)) - 1;
    for (int v = v0; v < 2 * v0 + 1; ++v) {
      const int p = v - v0, r = S[2 * v];
      if (d.enc == QUBIT) {  // CZ phase kickback from the routed cell
        if (S[2 * v + 1] && ((tb->mem[2 * p + r] >> fb) & 1u)) ph = -ph;
      } else if (r != 0) {  // computational-basis CNOT from the routed cell
        if ((tb->mem[2 * p + (r == 2 ? 1 : 0)] >> fb) & 1u) S[2 * v + 1] ^= 1;
      }
    }
  }
  const int sl = tb->store_l[s];
  if (sl >= 0) {
    for (int v = (1 << sl) - 1; v < (2 << sl) - 1; ++v) {
      int &r = S[2 * v], &x = S[2 * v + 1];
      if (d.enc == QUBIT) {
        swp(r, x);  // SWAP(a_v, d_v)
        continue;
      }
      // qutrit, gated by the parent's router: (W, b) <-> (L or R by b, 0)
      if (v > 0) {
        const int p = (v - 1) >> 1;
        if (S[2 * p] != ((v & 1) ? 1 : 2)) continue;
      }
      if (r == 0) {
        r = x ? 2 : 1;
        x = 0;
      } else if (x == 0) {
        x = r == 2 ? 1 : 0;
        r = 0;
      }
    }
  }
  return ph;
}

__global__ void k_zero(double2 *a, uint64_t m) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < m; i += (uint64_t)gridDim.x * blockDim.x)
    a[i] = make_double2(0.0, 0.0);
}

__global__ void k_put(double2 *a, const uint64_t *idx, const double2 *v, uint32_t m) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) a[idx[i]] = v[i];
}

// state vector: gates (a permutation with signs), scatter form
__global__ void k_psi_gates(const Tables *__restrict__ tb, const DDims d, int s, const double2 *in, double2 *out) {
  int g[DENSE_MAXD];
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < d.N; x += (uint64_t)gridDim.x * blockDim.x) {
    dec(d, x, g);
    const double ph = slice_gates(tb, d, s, g);
    const double2 u = in[x];
    out[enc_idx(d, g)] = make_double2(ph * u.x, ph * u.y);
  }
}

// Hadamard on bus bit b, in place over pairs
__global__ void k_psi_wall(const DDims d, int b, double2 *a) {
  const uint64_t pv = d.pv[d.n + b];
  const double h = 0.70710678118654752440;
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < d.N; x += (uint64_t)gridDim.x * blockDim.x) {
    if ((x / pv) & 1u) continue;
    const double2 u = a[x], v = a[x + pv];
    a[x] = make_double2(h * (u.x + v.x), h * (u.y + v.y));
    a[x + pv] = make_double2(h * (u.x - v.x), h * (u.y - v.y));
  }
}

// exp(2 pi i m / dd), exact for dd = 2 and to rounding for dd = 3
__device__ __forceinline__ double2 root_of_unity(int m, int dd) {
  m %= dd;
  if (m == 0) return make_double2(1.0, 0.0);
  if (dd == 2) return make_double2(-1.0, 0.0);
  return make_double2(-0.5, m == 1 ? 0.86602540378443864676 : -0.86602540378443864676);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Z^b X^a on site q: level v -> v + a, then the phase w^(b (v + a))
__global__ void k_psi_fault(const DDims d, int q, int fa, int fbz, const double2 *in, double2 *out) {
  const int di = d.n + d.k + q, dd = d.rad[di];
  const uint64_t pv = d.pv[di];
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < d.N; x += (uint64_t)gridDim.x * blockDim.x) {
    const int v = (int)((x / pv) % (uint64_t)dd), w = (v + fa) % dd;
    const uint64_t y = x + (uint64_t)(w - v) * pv;  // (unsigned wrap cancels)
    out[y] = cmul(root_of_unity(fbz * w, dd), in[x]);
  }
}

// K_J of Eq. layerkraus: J's sites must hold J's levels and are reset; the
// factor is sqrt(gamma)^|J| a^(excited sites - |J|)
__global__ void k_psi_kraus(const DDims d, const uint32_t *J, int nJ, double sg, double a, const double2 *in,
                            double2 *out) {
  int g[DENSE_MAXD];
  for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < d.N; x += (uint64_t)gridDim.x * blockDim.x) {
    dec(d, x, g);
    int *S = g + d.n + d.k;
    bool ok = true;
    for (int j = 0; j < nJ && ok; ++j) ok = S[J[j] & 0xFFFFu] == (int)((J[j] >> 16) & 0xFFu);
    if (!ok) continue;
    int ne = 0;
    for (int q = 0; q < d.M; ++q) ne += S[q] != 0;
    double f = 1.0;
    for (int j = 0; j < nJ; ++j) {
      f *= sg;
      S[J[j] & 0xFFFFu] = 0;
    }
    for (int e = 0; e < ne - nJ; ++e) f *= a;
    const double2 u = in[x];
    out[enc_idx(d, g)] = make_double2(f * u.x, f * u.y);
  }
}

// density matrix rho[x][y], row-major N x N
__global__ void k_rho_gates(const Tables *__restrict__ tb, const DDims d, int s, const double2 *in, double2 *out) {
  int gx[DENSE_MAXD], gy[DENSE_MAXD];
  const uint64_t NN = d.N * d.N;
  for (uint64_t z = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; z < NN; z += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t x = z / d.N, y = z % d.N;
    dec(d, x, gx);
    dec(d, y, gy);
    const double ph = slice_gates(tb, d, s, gx) * slice_gates(tb, d, s, gy);
    const double2 u = in[z];
    out[enc_idx(d, gx) * d.N + enc_idx(d, gy)] = make_double2(ph * u.x, ph * u.y);
  }
}

// Hadamard on bus bit b from the left (rows) or the right (columns)
__global__ void k_rho_wall(const DDims d, int b, int cols, double2 *r) {
  const uint64_t pv = d.pv[d.n + b], NN = d.N * d.N;
  const double h = 0.70710678118654752440;
  for (uint64_t z = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; z < NN; z += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t x = z / d.N, y = z % d.N, w = cols ? y : x;
    if ((w / pv) & 1u) continue;
    const uint64_t z1 = cols ? z + pv : z + pv * d.N;
    const double2 u = r[z], v = r[z1];
    r[z] = make_double2(h * (u.x + v.x), h * (u.y + v.y));
    r[z1] = make_double2(h * (u.x - v.x), h * (u.y - v.y));
  }
}

// The site channels on site q, gather form.  kind 0: depolarizing of
// strength p (uniform over the nontrivial Z^b X^a); 1: amplitude damping
// (every excited level decays to 0 with probability p); 2: dephasing
// ((1-p) rho + p Z rho Z+ on a qubit, (1-p) rho + (p/2) sum_{m=1,2} Z^m rho
// Z^m+ on a qutrit); 3: heating (level 0 rises with probability p, to 1 on a
// qubit, to 1 or 2 with p/2 each on a qutrit router; the no-jump operator is
// diag(sqrt(1-p), 1, 1)).
__global__ void k_rho_site(const DDims d, int q, int kind, double p, const double2 *in, double2 *out) {
  const int di = d.n + d.k + q, dd = d.rad[di];
  const uint64_t pv = d.pv[di], NN = d.N * d.N;
  for (uint64_t z = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; z < NN; z += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t x = z / d.N, y = z % d.N;
    const int vx = (int)((x / pv) % (uint64_t)dd), vy = (int)((y / pv) % (uint64_t)dd);
    const double2 u = in[z];
    double2 o;
    if (kind == 0) {
      const int nops = dd * dd - 1;
      o = make_double2((1.0 - p) * u.x, (1.0 - p) * u.y);
      const double c = p / nops;
      for (int fa = 0; fa < dd; ++fa)
        for (int fb = 0; fb < dd; ++fb) {
          if (fa == 0 && fb == 0) continue;
          // (U rho U+)[x][y] = w^(b x_q) conj(w^(b y_q)) rho[x - a][y - a]
          const int sx = (vx - fa + dd) % dd, sy = (vy - fa + dd) % dd;
          const double2 r = in[(x + (uint64_t)(sx - vx) * pv) * d.N + (y + (uint64_t)(sy - vy) * pv)];
          const double2 ph = root_of_unity(fb * (vx - vy + dd), dd);
          const double2 t = cmul(ph, r);
          o.x += c * t.x;
          o.y += c * t.y;
        }
    } else if (kind == 1) {
      const double a = sqrt(1.0 - p);
      const double f = (vx ? a : 1.0) * (vy ? a : 1.0);
      o = make_double2(f * u.x, f * u.y);
      if (vx == 0 && vy == 0)
        for (int lev = 1; lev < dd; ++lev) {
          const double2 r = in[(x + (uint64_t)lev * pv) * d.N + (y + (uint64_t)lev * pv)];
          o.x += p * r.x;
          o.y += p * r.y;
        }
    } else if (kind == 2) {
      const double f = vx == vy ? 1.0 : (dd == 2 ? 1.0 - 2.0 * p : 1.0 - 1.5 * p);
      o = make_double2(f * u.x, f * u.y);
    } else {
      const double a = sqrt(1.0 - p);
      const double f = (vx ? 1.0 : a) * (vy ? 1.0 : a);
      o = make_double2(f * u.x, f * u.y);
      if (vx != 0 && vx == vy) {
        const double c = dd == 2 ? p : 0.5 * p;
        const double2 r = in[(x - (uint64_t)vx * pv) * d.N + (y - (uint64_t)vy * pv)];
        o.x += c * r.x;
        o.y += c * r.y;
      }
    }
    out[z] = o;
  }
}

// <psi_id| rho |psi_id> over the ideal state's support, and the trace
__global__ void k_rho_measure(const DDims d, const double2 *r, const uint64_t *idx, const double2 *v, uint32_t m,
                              double *res) {
  double acc[3] = {0.0, 0.0, 0.0};
  const uint64_t mm = (uint64_t)m * m;
  for (uint64_t z = threadIdx.x; z < mm; z += blockDim.x) {
    const uint32_t i = (uint32_t)(z / m), j = (uint32_t)(z % m);
    const double2 a = v[i], b = v[j], rr = r[idx[i] * d.N + idx[j]];
    const double2 t = cmul(make_double2(a.x, -a.y), cmul(rr, b));
    acc[0] += t.x;
    acc[1] += t.y;
  }
  for (uint64_t x = threadIdx.x; x < d.N; x += blockDim.x) acc[2] += r[x * d.N + x].x;
  __shared__ double buf[16 * 3];
  block_sum<3>(acc, buf);
  if (threadIdx.x == 0) {
    res[0] = acc[0];
    res[1] = acc[2];
  }
}

DDims make_dims(int n, int k, int enc) {
  DDims d{};
  d.n = n;
  d.k = k;
  d.M = 2 * ((1 << n) - 1);
  d.enc = enc;
  d.nd = n + k + d.M;
  for (int i = 0; i < d.nd; ++i) {
    const int q = i - n - k;
    d.rad[i] = (q >= 0 && enc == QUTRIT && (q & 1) == 0) ? 3 : 2;
  }
  d.pv[d.nd - 1] = 1;
  for (int i = d.nd - 2; i >= 0; --i) d.pv[i] = d.pv[i + 1] * (uint64_t)d.rad[i + 1];
  d.N = d.pv[0] * (uint64_t)d.rad[0];
  return d;
}

uint64_t basis_index(const DDims &d, uint32_t i, uint32_t j) {
  uint64_t x = 0;
  for (int t = 0; t < d.n; ++t) x += (uint64_t)((i >> (d.n - 1 - t)) & 1u) * d.pv[t];
  for (int b = 0; b < d.k; ++b) x += (uint64_t)((j >> b) & 1u) * d.pv[d.n + b];
  return x;
}

int grid_for(uint64_t m) { return (int)std::min<uint64_t>((m + 255) / 256, 8192); }

#define DCHK(x)                          \
  do {                                   \
    hipError_t e_ = (x);                 \
    if (e_ != hipSuccess) return e_;     \
  } while (0)

// The active positions of slice s (App. C placement; R23): every site of
// the layers t < n-1 whose router holds its bit before and after slice s.
int active_sites(int n, int T, int s) {
  int l = 0;
  for (int t = 0; t + 1 < n; ++t)
    if (3 * t + 2 < s && s < T - 3 * t - 2) ++l;
  return 2 * ((1 << l) - 1);
}

}  // namespace

uint64_t dense_dim(int n, int k, int enc) { return make_dims(n, k, enc).N; }

hipError_t dense_density(const Tables *dtab, const DenseJob &job, hipStream_t st, double *F, double *tr) {
  const DDims d = make_dims(job.n, job.k, job.enc);
  const uint64_t NN = d.N * d.N;
  const int T = 6 * job.n + 2 * job.k;
  double2 *r0 = nullptr, *r1 = nullptr, *v = nullptr;
  uint64_t *ix = nullptr;
  double *res = nullptr;
  const uint32_t m = (uint32_t)job.in_idx.size();
  hipError_t e = hipSuccess;
  auto cleanup = [&]() {
    (void)hipFree(r0);
    (void)hipFree(r1);
    (void)hipFree(v);
    (void)hipFree(ix);
    (void)hipFree(res);
  };
  auto run = [&]() -> hipError_t {
    DCHK(hipMalloc(&r0, NN * sizeof(double2)));
    DCHK(hipMalloc(&r1, NN * sizeof(double2)));
    DCHK(hipMalloc(&v, std::max<size_t>(m, 1) * sizeof(double2)));
    DCHK(hipMalloc(&ix, std::max<size_t>(m, 1) * sizeof(uint64_t)));
    DCHK(hipMalloc(&res, 2 * sizeof(double)));
    // rho = |psi0><psi0| over the input's support
    std::vector<uint64_t> hx(m);
    std::vector<double2> hv(m);
    for (uint32_t t = 0; t < m; ++t) {
      hx[t] = basis_index(d, job.in_idx[t] >> 8, job.in_idx[t] & 0xFFu);
      hv[t] = make_double2(job.in_amp[2 * t], job.in_amp[2 * t + 1]);
    }
    std::vector<uint64_t> pairs_i;
    std::vector<double2> pairs_v;
    for (uint32_t a = 0; a < m; ++a)
      for (uint32_t b = 0; b < m; ++b) {
        pairs_i.push_back(hx[a] * d.N + hx[b]);
        const double2 x = hv[a], y = hv[b];  // psi[a] conj(psi[b])
        pairs_v.push_back(make_double2(x.x * y.x + x.y * y.y, x.y * y.x - x.x * y.y));
      }
    uint64_t *pi = nullptr;
    double2 *pvv = nullptr;
    DCHK(hipMalloc(&pi, std::max<size_t>(pairs_i.size(), 1) * sizeof(uint64_t)));
    DCHK(hipMalloc(&pvv, std::max<size_t>(pairs_v.size(), 1) * sizeof(double2)));
    hipError_t e2 = hipMemcpy(pi, pairs_i.data(), pairs_i.size() * 8, hipMemcpyHostToDevice);
    if (e2 == hipSuccess) e2 = hipMemcpy(pvv, pairs_v.data(), pairs_v.size() * 16, hipMemcpyHostToDevice);
    if (e2 == hipSuccess) {
      k_zero<<<grid_for(NN), 256, 0, st>>>(r0, NN);
      k_put<<<(uint32_t)((pairs_i.size() + 255) / 256), 256, 0, st>>>(r0, pi, pvv, (uint32_t)pairs_i.size());
      e2 = hipStreamSynchronize(st);
    }
    (void)hipFree(pi);
    (void)hipFree(pvv);
    DCHK(e2);
    if (job.enc == QUBIT)
      for (int b = 0; b < job.k; ++b) {
        k_rho_wall<<<grid_for(NN), 256, 0, st>>>(d, b, 0, r0);
        k_rho_wall<<<grid_for(NN), 256, 0, st>>>(d, b, 1, r0);
      }
    for (int s = 1; s < T; ++s) {
      k_rho_gates<<<grid_for(NN), 256, 0, st>>>(dtab, d, s, r0, r1);
      std::swap(r0, r1);
      if (job.eps > 0.0)
        for (int q = 0; q < active_sites(job.n, T, s); ++q) {
          k_rho_site<<<grid_for(NN), 256, 0, st>>>(d, q, 0, job.eps, r0, r1);
          std::swap(r0, r1);
        }
      const double ps[3] = {job.gamma, job.dephase, job.heat};
      for (int kind = 1; kind <= 3; ++kind) {
        if (ps[kind - 1] <= 0.0) continue;
        for (int q = 0; q < d.M; ++q) {
          k_rho_site<<<grid_for(NN), 256, 0, st>>>(d, q, kind, ps[kind - 1], r0, r1);
          std::swap(r0, r1);
        }
      }
    }
    if (job.enc == QUBIT)
      for (int b = 0; b < job.k; ++b) {
        k_rho_wall<<<grid_for(NN), 256, 0, st>>>(d, b, 0, r0);
        k_rho_wall<<<grid_for(NN), 256, 0, st>>>(d, b, 1, r0);
      }
    // the ideal output sum_ij c_ij |i>|j xor d_i>|ground>
    for (uint32_t t = 0; t < m; ++t) {
      const uint32_t i = job.in_idx[t] >> 8, j = job.in_idx[t] & 0xFFu;
      hx[t] = basis_index(d, i, j ^ (job.mem[i] & ((1u << job.k) - 1u)));
    }
    DCHK(hipMemcpy(ix, hx.data(), m * 8, hipMemcpyHostToDevice));
    DCHK(hipMemcpy(v, hv.data(), m * 16, hipMemcpyHostToDevice));
    k_rho_measure<<<1, 256, 0, st>>>(d, r0, ix, v, m, res);
    double hres[2];
    DCHK(hipMemcpyAsync(hres, res, 16, hipMemcpyDeviceToHost, st));
    DCHK(hipStreamSynchronize(st));
    *F = hres[0];
    *tr = hres[1];
    return hipGetLastError();
  };
  e = run();
  cleanup();
  return e;
}

hipError_t dense_forced(const Tables *dtab, const DenseJob &job, const uint32_t *jumps, uint32_t njumps,
                        const uint32_t *faults, uint32_t nfaults, hipStream_t st, double *psi_host) {
  const DDims d = make_dims(job.n, job.k, job.enc);
  const int T = 6 * job.n + 2 * job.k;
  double2 *p0 = nullptr, *p1 = nullptr, *v = nullptr;
  uint64_t *ix = nullptr;
  uint32_t *dj = nullptr;
  const uint32_t m = (uint32_t)job.in_idx.size();
  auto run = [&]() -> hipError_t {
    DCHK(hipMalloc(&p0, d.N * sizeof(double2)));
    DCHK(hipMalloc(&p1, d.N * sizeof(double2)));
    DCHK(hipMalloc(&v, std::max<size_t>(m, 1) * sizeof(double2)));
    DCHK(hipMalloc(&ix, std::max<size_t>(m, 1) * sizeof(uint64_t)));
    DCHK(hipMalloc(&dj, JMAX * sizeof(uint32_t)));
    std::vector<uint64_t> hx(m);
    std::vector<double2> hv(m);
    for (uint32_t t = 0; t < m; ++t) {
      hx[t] = basis_index(d, job.in_idx[t] >> 8, job.in_idx[t] & 0xFFu);
      hv[t] = make_double2(job.in_amp[2 * t], job.in_amp[2 * t + 1]);
    }
    DCHK(hipMemcpy(ix, hx.data(), m * 8, hipMemcpyHostToDevice));
    DCHK(hipMemcpy(v, hv.data(), m * 16, hipMemcpyHostToDevice));
    k_zero<<<grid_for(d.N), 256, 0, st>>>(p0, d.N);
    k_put<<<(m + 255) / 256, 256, 0, st>>>(p0, ix, v, m);
    if (job.enc == QUBIT)
      for (int b = 0; b < job.k; ++b) k_psi_wall<<<grid_for(d.N), 256, 0, st>>>(d, b, p0);
    const double sg = std::sqrt(job.gamma), a = std::sqrt(1.0 - job.gamma);
    uint32_t jpos = 0, fpos = 0;
    for (int s = 1; s < T; ++s) {
      k_psi_gates<<<grid_for(d.N), 256, 0, st>>>(dtab, d, s, p0, p1);
      std::swap(p0, p1);
      for (; fpos < nfaults && (int)((faults[fpos] >> 16) & 0xFFu) == s; ++fpos) {
        const uint32_t f = faults[fpos], ty = f >> 24;
        k_psi_fault<<<grid_for(d.N), 256, 0, st>>>(d, (int)(f & 0xFFFFu), (int)(ty & 3u), (int)(ty >> 2), p0, p1);
        std::swap(p0, p1);
      }
      uint32_t hJ[JMAX];
      int nJ = 0;
      for (; jpos < njumps && (int)(jumps[jpos] >> 24) == s; ++jpos)
        if (nJ < JMAX) hJ[nJ++] = jumps[jpos] & 0xFFFFFFu;
      if (nJ) DCHK(hipMemcpyAsync(dj, hJ, nJ * 4, hipMemcpyHostToDevice, st));
      k_zero<<<grid_for(d.N), 256, 0, st>>>(p1, d.N);
      k_psi_kraus<<<grid_for(d.N), 256, 0, st>>>(d, dj, nJ, sg, a, p0, p1);
      std::swap(p0, p1);
      DCHK(hipStreamSynchronize(st));  // (hJ is reused)
    }
    DCHK(hipMemcpyAsync(psi_host, p0, d.N * sizeof(double2), hipMemcpyDeviceToHost, st));
    DCHK(hipStreamSynchronize(st));
    return hipGetLastError();
  };
  const hipError_t e = run();
  (void)hipFree(p0);
  (void)hipFree(p1);
  (void)hipFree(v);
  (void)hipFree(ix);
  (void)hipFree(dj);
  return e;
}

}  // namespace qr
