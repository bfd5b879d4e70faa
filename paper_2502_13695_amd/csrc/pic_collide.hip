// Binary Coulomb collisions among the charged macroparticles (gfx950).
//
// The paper (Sec. 2.2, Eq. 4) collides all charged particles with the
// Perez/Nanbu binary model of its host code: collision frequency
// nu = (q_a q_b)^2 n_b ln(Lambda) / (4 pi (eps0 mu)^2) / v_r^3, the Coulomb
// logarithm computed per collision with a lower bound of 1, and a
// low-temperature extension.  The published method it names (Perez et al.
// 2012, Nanbu 1997, Nanbu & Yonemura 1998) is restated here:
//
// * per step, after ionization, the particles are binned by cell (count,
//   scan, fill), and each cell's entries ordered by (kind, Philox key, id);
//   the order does not depend on where the particles sit in memory;
// * one thread per cell runs the cell's collisions in a fixed sequence: each
//   kind with itself (pairs of consecutive entries; an odd count first forms
//   a triangle of three half-strength collisions), kinds ascending, then each
//   pair of kinds a < b (collision i takes the (i mod Na)-th of a and the
//   (i mod Nb)-th of b), each collision reading the momenta the previous left;
// * per collision: the centre-of-momentum frame, the scattering parameter s
//   (whose non-relativistic limit is nu dt of Eq. 4), the cap of one mean free
//   path, the deflection angle from Nanbu's law through Perez's fit of A(s),
//   a uniform azimuth, back to the lab frame; unlike weights follow Nanbu and
//   Yonemura's rule (update with probability w_other / w_max).
// The arithmetic is FP64; momenta are stored back as FP32.

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>

#include "pic_kernels.h"

namespace pic {

namespace {

constexpr uint32_t PURPOSE_PAIR = 7, PURPOSE_SCATTER = 8, PURPOSE_IMPACT = 9;
constexpr double kC = 299792458.0, kEPS0 = 8.8541878128e-12, kHBAR = 1.054571817e-34,
                 kQE = 1.602176634e-19, kPI = 3.14159265358979323846;
constexpr int SCAN_B = COL_SCAN_B;

__device__ __forceinline__ int box_cell(const Inst& I, uint32_t pc) {
  int i, j, k;
  unpack_cell(I.D, pc, i, j, k);
  return i + I.nx * (j + I.ny * k);
}

__device__ __forceinline__ int live_slots(const Inst& I) {
  const int n = *I.pcount;
  return n < I.capacity ? n : I.capacity;
}

__global__ void k_col_clear(ColBufs b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= b.ncell) b.cnt[i] = 0;
  if (i < b.ncell) b.fill[i] = 0;
}

// counts per cell (no return value is waited for)
__global__ void k_col_count(const Inst I, ColBufs b) {
  const int n = live_slots(I);
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x)
    if (I.pkind[p] != 0xFF) atomicAdd(&b.cnt[box_cell(I, I.pcell[p])], 1);
}

// exclusive scan of v over a block of SCAN_B threads (a scan within each
// wave, then over the wave totals); the block's total in *total.  w holds
// SCAN_B / 64 + 1 ints of LDS.
__device__ __forceinline__ int block_scan(int v, int* w, int* total) {
  constexpr int NW = SCAN_B / 64;
  const int lane = (int)__lane_id(), wv = threadIdx.x / 64;
  int x = v;
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) w[wv] = x;
  __syncthreads();
  if (wv == 0) {
    const int s0 = lane < NW ? w[lane] : 0;
    int y = s0;
    for (int off = 1; off < NW; off <<= 1) {
      const int z = __shfl_up(y, off);
      if (lane >= off) y += z;
    }
    if (lane < NW) w[lane] = y - s0;
    if (lane == NW - 1) w[NW] = y;
  }
  __syncthreads();
  const int r = w[wv] + x - v;
  *total = w[NW];
  __syncthreads();
  return r;
}

// exclusive scan of cnt[0 .. n): per block, block totals, then offsets.  The
// local pass also lists the cells that have work, ascending, at the front of
// the block's segment of active: a cell of a material with impact ionization
// holding a particle, else any cell holding two when collisions are on.
__global__ __launch_bounds__(SCAN_B) void k_col_scan_local(const Inst I, ColBufs b, int n) {
  __shared__ int w[SCAN_B / 64 + 1];
  const int c = blockIdx.x * SCAN_B + threadIdx.x;
  const int cnt = c < n ? b.cnt[c] : 0;
  bool list = false;
  if (cnt > 0) {
    bool imp = false;
    if (b.impact) {
      const int m = I.mat_cell[c % I.nx];
      imp = m >= 0 && b.imp_P[m] > 0.0;
    }
    list = imp || (b.collide && cnt >= 2);
  }
  int tot;
  const int off = block_scan(cnt, w, &tot);
  if (c < n) b.cnt[c] = off;
  if (threadIdx.x == 0) b.bsum[blockIdx.x] = tot;
  const int r = block_scan(list ? 1 : 0, w, &tot);
  if (list) b.active[blockIdx.x * SCAN_B + r] = c;
  if (threadIdx.x == 0) b.bact[blockIdx.x] = tot;
}

// one block: exclusive scans of the block totals (bsum) and of the blocks'
// listed cells (bact, whose entry nb takes the total), each thread a chunk
__global__ __launch_bounds__(SCAN_B) void k_col_scan_top(ColBufs b, int nb) {
  __shared__ int w[SCAN_B / 64 + 1];
  const int per = (nb + SCAN_B - 1) / SCAN_B;
  const int t0 = threadIdx.x * per;
  for (int a = 0; a < 2; ++a) {
    int* v = a ? b.bact : b.bsum;
    int sum = 0;
    for (int q = 0; q < per; ++q)
      if (t0 + q < nb) sum += v[t0 + q];
    int tot;
    int run = block_scan(sum, w, &tot);
    for (int q = 0; q < per; ++q)
      if (t0 + q < nb) {
        const int x = v[t0 + q];
        v[t0 + q] = run;
        run += x;
      }
    if (a && threadIdx.x == 0) v[nb] = tot;
  }
}

// offsets of the blocks added; each block's listed cells gathered into list
__global__ __launch_bounds__(SCAN_B) void k_col_scan_add(ColBufs b, int n) {
  const int i = blockIdx.x * SCAN_B + threadIdx.x;
  if (i < n) b.cnt[i] += b.bsum[blockIdx.x];
  const int a0 = b.bact[blockIdx.x], na = b.bact[blockIdx.x + 1] - a0;
  if ((int)threadIdx.x < na) b.list[a0 + threadIdx.x] = b.active[i];
}

__global__ void k_col_fill(const Inst I, ColBufs b, int step) {
  const int n = live_slots(I);
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
    const uint8_t kd = I.pkind[p];
    if (kd == 0xFF) continue;
    const int c = box_cell(I, I.pcell[p]);
    const int q = b.cnt[c] + atomicAdd(&b.fill[c], 1);
    b.idx[q] = p;
    b.key[q] = (uint64_t)kd << 32 | draw(I.seed, (uint64_t)I.pid[p] | ((uint64_t)kd << 32), (uint32_t)step, PURPOSE_PAIR).x;
  }
}

struct D3 {
  double x, y, z;
};
__device__ __forceinline__ D3 operator+(D3 a, D3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ D3 operator*(double s, D3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ double dot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

__device__ __forceinline__ double unif(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

// Nanbu's deflection: <cos chi> = coth A - 1/A = exp(-s); Perez's fit of 1/A
// on 0.1 <= s < 3, the small-angle law below, A = 3 exp(-s) up to 6, isotropic
// above.  FP64: small deflections take sin(chi) from 1 - cos(chi), which FP32
// would leave with a few digits only.
__device__ double cos_chi(double s, double U) {
  // one exp(-s), one division, one exp(A) and one log per lane whatever its
  // range, so that lanes of a wave in different ranges do not run each
  // range's transcendentals in turn (same operations per range as written out)
  const bool small = s < 0.1, fit = s < 3.0;
  const double poly = 0.0056958 + s * (0.9560202 + s * (-0.508139 + s * (0.47913906 + s * (-0.12788975 + s * 0.02389567))));
  const double e3 = fit ? 1.0 : 3.0 * exp(-s);
  const double d = fit ? poly : e3;
  const double r = 1.0 / d;
  const double ainv = fit ? poly : r, A = fit ? r : e3;
  const double eA = small || s >= 6.0 ? 1.0 : exp(A);
  const double arg = small ? U : (1.0 - U) / eA + U * eA;
  const double L = log(arg);
  if (small) return fmax(-1.0, 1.0 + s * L);
  if (s < 6.0) return fmin(1.0, fmax(-1.0, ainv * L));
  return 2.0 * U - 1.0;
}

// what the impact pass writes besides the momenta: neutrals and births
struct ImpView {
  uint32_t* alive;
  int* death;
  const float *no0, *no1, *no2;
  uint32_t* pcell;
  uint32_t *po0, *po1, *po2;
  uint8_t* pkind;
  int* pcount;
  unsigned* health;
  unsigned long long* nevents;
  const float* ksig;
  const signed char* mat_cell;
  int capacity, D, nx, ny, ppc;
};

// what a collision reads and writes (the kinds' masses and weights in LDS)
struct PView {
  float *u0, *u1, *u2;
  uint32_t* pid;
  uint64_t seed;
  const double* mass;
  const double* w;
};

// One collision of entries a (kind ka) and b (kind kb); updates the slots'
// momenta.  ld: the cell's Debye length (0: none); mn13: the larger m n^(-1/3)
// of the two kinds (the low-temperature cap); n: the density in s.
__device__ __forceinline__ void collide_pair(const PView& I, double ld, double mn13, double dt, int pa, int pb, int ka,
                                             int kb, double n, bool half, uint32_t r, int step) {
  const double m1 = I.mass[ka], m2 = I.mass[kb];
  const double q1 = (ka & 1) ? kQE : -kQE, q2 = (kb & 1) ? kQE : -kQE;
  const D3 u1{I.u0[pa], I.u1[pa], I.u2[pa]};
  const D3 u2{I.u0[pb], I.u1[pb], I.u2[pb]};
  const double g1 = sqrt(1.0 + dot(u1, u1)), g2 = sqrt(1.0 + dot(u2, u2));
  const D3 bc = (1.0 / (m1 * g1 + m2 * g2)) * (m1 * u1 + m2 * u2);
  const double bc2 = dot(bc, bc);
  const double gc = 1.0 / sqrt(1.0 - bc2);
  const D3 b1 = (1.0 / g1) * u1, b2 = (1.0 / g2) * u2;
  D3 p1s;   // particle 1's momentum in the centre-of-momentum frame [kg m/s]
  if (bc2 > 0.0)
    p1s = (m1 * kC) * (u1 + (((gc - 1.0) / bc2 * dot(bc, b1) - gc) * g1) * bc);
  else
    p1s = (m1 * kC) * u1;
  const double g1s = gc * g1 * (1.0 - dot(bc, b1));
  const double g2s = gc * g2 * (1.0 - dot(bc, b2));
  const double P = sqrt(dot(p1s, p1s));
  if (P == 0.0) return;
  const double mu = m1 * m2 / (m1 + m2);
  const double v1s = P / (m1 * g1s), v2s = P / (m2 * g2s);
  const double vrel = (v1s + v2s) / (1.0 + v1s * v2s / (kC * kC));
  double lnL = 1.0;
  if (ld > 0.0) {
    const double bcl = fabs(q1 * q2) / (4.0 * kPI * kEPS0 * mu * vrel * vrel);
    const double bqm = kHBAR / (2.0 * mu * vrel);
    lnL = fmax(1.0, log(ld / fmax(bcl, bqm)));
  }
  const double f = m1 * g1s * m2 * g2s * kC * kC / (P * P) + 1.0;
  double s = n * dt * lnL * (q1 * q2) * (q1 * q2) /
             (4.0 * kPI * kEPS0 * kEPS0 * kC * kC * kC * kC * m1 * g1 * m2 * g2) * gc * P / (m1 * g1 + m2 * g2) * f * f;
  const double cap = 1.6119919540164696 * dt * (m1 + m2) * vrel / mn13;   // (4 pi / 3)^(1/3)
  s = fmin(s, cap);
  if (half) s *= 0.5;
  const uint32_t hi = (uint32_t)ka | ((uint32_t)kb << 8) | (r << 16);
  const u32x4 w = draw(I.seed, (uint64_t)I.pid[pa] | ((uint64_t)hi << 32), (uint32_t)step, PURPOSE_SCATTER);
  const double cchi = cos_chi(s, unif(w.x));
  const double schi = sqrt(fmax(0.0, 1.0 - cchi * cchi));
  float sphf, cphf;
  sincosf(6.2831853071795865f * (float)unif(w.y), &sphf, &cphf);
  const double sphi = sphf, cphi = cphf;
  const double pperp = sqrt(p1s.x * p1s.x + p1s.y * p1s.y);
  D3 q;
  if (pperp > 0.0) {
    q = {p1s.x * p1s.z / pperp * schi * cphi - p1s.y * P / pperp * schi * sphi + p1s.x * cchi,
         p1s.y * p1s.z / pperp * schi * cphi + p1s.x * P / pperp * schi * sphi + p1s.y * cchi,
         -pperp * schi * cphi + p1s.z * cchi};
  } else {
    q = {P * schi * cphi, P * schi * sphi, p1s.z * cchi};
  }
  D3 p1n, p2n;
  if (bc2 > 0.0) {
    const double fq = (gc - 1.0) / bc2 * dot(bc, q);
    p1n = q + (fq + m1 * kC * g1s * gc) * bc;
    p2n = (-1.0) * q + (-fq + m2 * kC * g2s * gc) * bc;
  } else {
    p1n = q;
    p2n = (-1.0) * q;
  }
  const double w1 = I.w[ka], w2 = I.w[kb], wmax = fmax(w1, w2);
  const double U3 = unif(w.z);
  if (U3 < w2 / wmax) {
    const double sc = 1.0 / (m1 * kC);
    I.u0[pa] = (float)(sc * p1n.x);
    I.u1[pa] = (float)(sc * p1n.y);
    I.u2[pa] = (float)(sc * p1n.z);
  }
  if (U3 < w1 / wmax) {
    const double sc = 1.0 / (m2 * kC);
    I.u0[pb] = (float)(sc * p2n.x);
    I.u1[pb] = (float)(sc * p2n.y);
    I.u2[pb] = (float)(sc * p2n.z);
  }
}

// entry order inside a cell: (kind, key, id), the first two in one word
__device__ __forceinline__ bool before(const uint32_t* pid, uint64_t ka, int pa, uint64_t kb, int pb) {
  if (ka != kb) return ka < kb;
  return pid[pa] < pid[pb];
}

// Impact ionization in cell c (its entries ordered): each electron of the
// cell's material decides once; an event takes the cell's alive neutral of
// lowest index, the electron pays the gap, the pair is born at the neutral.
__device__ __forceinline__ void impact_cell(const ColBufs& b, const PView& pv, const ImpView& v, const uint8_t* kind,
                            const double* smass, int c, int e0, int e1, int step) {
  const int i = c % v.nx, j = (c / v.nx) % v.ny, k = c / (v.nx * v.ny);
  const int m = v.mat_cell[i];
  if (m < 0 || !(b.imp_P[m] > 0.0)) return;
  const int64_t j0 = ((int64_t)(j + v.ny * k) * b.nmx + b.mrank[i]) * v.ppc;
  int next = 0;   // neutrals below it are dead or taken
  for (int a = e0; a < e1; ++a) {
    const int p = b.idx[a];
    const int kd = kind[p];
    if (kd != 2 * m) continue;
    const double ux = pv.u0[p], uy = pv.u1[p], uz = pv.u2[p];
    const double uu = ux * ux + uy * uy + uz * uz;
    const double mc2 = smass[kd] * kC * kC;
    const double ke = (sqrt(1.0 + uu) - 1.0) * mc2;
    const double x = ke / b.imp_th[m] - 1.0;
    if (!(x > 0.0)) continue;
    const double prob = -expm1(-b.imp_P[m] * x * x * b.dt);
    const uint32_t w = draw(pv.seed, (uint64_t)pv.pid[p] | ((uint64_t)kd << 32), (uint32_t)step, PURPOSE_IMPACT).x;
    if (!((double)w + 0.5 < prob * 4294967296.0)) continue;
    while (next < v.ppc && !((v.alive[(j0 + next) >> 5] >> ((j0 + next) & 31)) & 1u)) ++next;
    if (next >= v.ppc) continue;
    const int64_t jn = j0 + next;
    const uint64_t id = (uint64_t)c * (uint64_t)v.ppc + (uint64_t)next;
    ++next;
    atomicAnd(&v.alive[jn >> 5], ~(1u << (jn & 31)));
    v.death[jn] = step;
    atomicAdd(&v.nevents[(blockIdx.x & 7) * 32 + m], 1ull);
    // the impacting electron pays the gap, direction kept
    const double g2 = 1.0 + (ke - b.gap[m]) / mc2;
    const double sc = sqrt(g2 * g2 - 1.0) / sqrt(uu);
    pv.u0[p] = (float)(sc * ux);
    pv.u1[p] = (float)(sc * uy);
    pv.u2[p] = (float)(sc * uz);
    const int q = atomicAdd(v.pcount, 2);
    if (q + 2 > v.capacity) {
      atomicOr(v.health, HEALTH_CAPACITY);
      continue;
    }
    float bx, by, bz;
    maxwell(pv.seed, id, PURPOSE_VEL, v.ksig[m], bx, by, bz);
    const uint32_t pc = pack_cell(v.D, i, j, k);
    for (int s = 0; s < 2; ++s) {
      v.pcell[q + s] = pc;
      v.po0[q + s] = off_fix(v.no0[jn]);
      if (v.D >= 2) v.po1[q + s] = off_fix(v.no1[jn]);
      if (v.D >= 3) v.po2[q + s] = off_fix(v.no2[jn]);
      pv.u0[q + s] = bx;
      pv.u1[q + s] = by;
      pv.u2[q + s] = bz;
      v.pkind[q + s] = (uint8_t)(2 * m + s);
      pv.pid[q + s] = (uint32_t)id;
    }
  }
}

__device__ __noinline__ void collide_sorted_any(const int* idx, int nk, double dt, PView pv, const uint8_t* kind,
                                                double vcell, int e0, int e1, int step);
__device__ __forceinline__ bool collide_groups(const ColBufs& b, const PView& pv, const uint8_t* kind, double vcell,
                                               const double* smass, const double* sw, int e0, int e1, int step);

constexpr int SORT_LDS = 16;    // entries of a cell sorted in LDS (larger cells: in place)
constexpr int CELLS_TPB = 256;  // threads per block of the cell pass

// the collisions (at least two particles) and the impact ionization of one
// cell; sk / si: this thread's SORT_LDS LDS entries, stride CELLS_TPB
__device__ __forceinline__ void collide_cell(const ColBufs& b, const PView& pv, const ImpView& iv, const uint8_t* kind,
                                             double vcell, const double* smass, const double* sw, uint64_t* sk,
                                             int* si, int c, int step) {
  const int e0 = b.cnt[c], e1 = b.cnt[c + 1];
  const int n = e1 - e0;
  constexpr int st = CELLS_TPB;
  // insertion sort of the cell's entries
  if (n <= SORT_LDS) {
    for (int a = 0; a < n; ++a) {
      sk[a * st] = b.key[e0 + a];
      si[a * st] = b.idx[e0 + a];
    }
    for (int a = 1; a < n; ++a) {
      const int p = si[a * st];
      const uint64_t k = sk[a * st];
      int j = a - 1;
      while (j >= 0 && before(pv.pid, k, p, sk[j * st], si[j * st])) {
        si[(j + 1) * st] = si[j * st];
        sk[(j + 1) * st] = sk[j * st];
        --j;
      }
      si[(j + 1) * st] = p;
      sk[(j + 1) * st] = k;
    }
    for (int a = 0; a < n; ++a) b.idx[e0 + a] = si[a * st];
  } else {
    for (int a = e0 + 1; a < e1; ++a) {
      const int p = b.idx[a];
      const uint64_t k = b.key[a];
      int j = a - 1;
      while (j >= e0 && before(pv.pid, k, p, b.key[j], b.idx[j])) {
        b.idx[j + 1] = b.idx[j];
        b.key[j + 1] = b.key[j];
        --j;
      }
      b.idx[j + 1] = p;
      b.key[j + 1] = k;
    }
  }
  if (b.collide && e1 - e0 >= 2 && !collide_groups(b, pv, kind, vcell, smass, sw, e0, e1, step))
    collide_sorted_any(b.idx, b.nk, b.dt, pv, kind, vcell, e0, e1, step);
  if (b.impact) impact_cell(b, pv, iv, kind, smass, c, e0, e1, step);
}

// The collisions of a cell's ordered entries [e0, e1), any number of kinds:
// per-kind tables (kept in scratch).  Cells with at most GMAX kinds take
// collide_groups below, which gives the same results.
__device__ __noinline__ void collide_sorted_any(const int* idx, int nk, double dt, PView pv, const uint8_t* kind,
                                                double vcell, int e0, int e1, int step) {
  const double* smass = pv.mass;
  const double* sw = pv.w;
  // kinds present: their entry ranges, densities and temperatures
  int kfirst[MAXKIND], kcount[MAXKIND];
  double dens[MAXKIND], mn13[MAXKIND], ke[MAXKIND];
  for (int k = 0; k < nk; ++k) {
    kcount[k] = 0;
    kfirst[k] = 0;
    dens[k] = 0.0;
    ke[k] = 0.0;
  }
  for (int a = e0; a < e1; ++a) {
    const int p = idx[a];
    const int k = kind[p];
    if (kcount[k] == 0) kfirst[k] = a;
    ++kcount[k];
    const double ux = pv.u0[p], uy = pv.u1[p], uz = pv.u2[p];
    ke[k] += (sqrt(1.0 + (ux * ux + uy * uy + uz * uz)) - 1.0) * smass[k] * kC * kC;
  }
  double inv_ld2 = 0.0;
  for (int k = 0; k < nk; ++k) {
    mn13[k] = 0.0;
    if (!kcount[k]) continue;
    dens[k] = kcount[k] * sw[k] / vcell;
    mn13[k] = smass[k] / cbrt(dens[k]);
    const double T = 2.0 / 3.0 * ke[k] / kcount[k];
    if (T > 0.0) inv_ld2 += dens[k] * kQE * kQE / (kEPS0 * T);
  }
  const double ld = inv_ld2 > 0.0 ? 1.0 / sqrt(inv_ld2) : 0.0;
  // like kinds
  for (int k = 0; k < nk; ++k) {
    const int N = kcount[k];
    if (N < 2) continue;
    const int f = kfirst[k];
    const double n = dens[k], m = mn13[k];
    int start = 0;
    if (N & 1) {
      collide_pair(pv, ld, m, dt, idx[f], idx[f + 1], k, k, n, true, 0, step);
      collide_pair(pv, ld, m, dt, idx[f + 1], idx[f + 2], k, k, n, true, 0, step);
      collide_pair(pv, ld, m, dt, idx[f + 2], idx[f], k, k, n, true, 0, step);
      start = 3;
    }
    for (int a = start; a + 1 < N; a += 2) collide_pair(pv, ld, m, dt, idx[f + a], idx[f + a + 1], k, k, n, false, 0, step);
  }
  // unlike kinds
  for (int ka = 0; ka < nk; ++ka) {
    if (!kcount[ka]) continue;
    for (int kb = ka + 1; kb < nk; ++kb) {
      if (!kcount[kb]) continue;
      const int Na = kcount[ka], Nb = kcount[kb];
      const int nmin = Na < Nb ? Na : Nb, nmax = Na < Nb ? Nb : Na;
      const double n = nmin * fmax(sw[ka], sw[kb]) / vcell, m = fmax(mn13[ka], mn13[kb]);
      for (int i = 0; i < nmax; ++i)
        collide_pair(pv, ld, m, dt, idx[kfirst[ka] + i % Na], idx[kfirst[kb] + i % Nb], ka, kb, n, false,
                     (uint32_t)(i / nmin), step);
    }
  }
}

constexpr int GMAX = 4;   // kinds of a cell whose tables stay in registers

// a[g] for a wave-varying g, as a chain of selects (keeps a in registers)
template <typename T>
__device__ __forceinline__ T pick(const T (&a)[GMAX], int g) {
  T r = a[0];
#pragma unroll
  for (int i = 1; i < GMAX; ++i) r = g == i ? a[i] : r;
  return r;
}

// The collisions of a cell's ordered entries [e0, e1) holding at most GMAX
// kinds: the kinds present form groups of consecutive entries, ascending; the
// sequence, densities, temperatures and sums are those of collide_sorted_any.
// Returns false, having changed nothing, for a cell with more kinds.
__device__ __forceinline__ bool collide_groups(const ColBufs& b, const PView& pv, const uint8_t* kind, double vcell,
                                               const double* smass, const double* sw, int e0, int e1, int step) {
  int gk[GMAX], gf[GMAX], gn[GMAX];
  double gke[GMAX];
#pragma unroll
  for (int g = 0; g < GMAX; ++g) {
    gk[g] = 0;
    gf[g] = 0;
    gn[g] = 0;
    gke[g] = 0.0;
  }
  int G = 0, last = -1;
  for (int a = e0; a < e1; ++a) {
    const int p = b.idx[a];
    const int k = kind[p];
    if (k != last) {
      if (G == GMAX) return false;
#pragma unroll
      for (int g = 0; g < GMAX; ++g)
        if (g == G) {
          gk[g] = k;
          gf[g] = a;
        }
      ++G;
      last = k;
    }
    const double ux = pv.u0[p], uy = pv.u1[p], uz = pv.u2[p];
    const double e = (sqrt(1.0 + (ux * ux + uy * uy + uz * uz)) - 1.0) * smass[k] * kC * kC;
#pragma unroll
    for (int g = 0; g < GMAX; ++g)
      if (g == G - 1) {
        ++gn[g];
        gke[g] += e;
      }
  }
  double dens[GMAX], mn13[GMAX];
  double inv_ld2 = 0.0;
#pragma unroll
  for (int g = 0; g < GMAX; ++g) {
    dens[g] = 0.0;
    mn13[g] = 0.0;
    if (g < G) {
      const int k = gk[g];
      dens[g] = gn[g] * sw[k] / vcell;
      mn13[g] = smass[k] / cbrt(dens[g]);
      const double T = 2.0 / 3.0 * gke[g] / gn[g];
      if (T > 0.0) inv_ld2 += dens[g] * kQE * kQE / (kEPS0 * T);
    }
  }
  const double ld = inv_ld2 > 0.0 ? 1.0 / sqrt(inv_ld2) : 0.0;
  // like kinds
  for (int g = 0; g < G; ++g) {
    const int N = pick(gn, g);
    if (N < 2) continue;
    const int k = pick(gk, g), f = pick(gf, g);
    const double n = pick(dens, g), m = pick(mn13, g);
    int start = 0;
    if (N & 1) {
      collide_pair(pv, ld, m, b.dt, b.idx[f], b.idx[f + 1], k, k, n, true, 0, step);
      collide_pair(pv, ld, m, b.dt, b.idx[f + 1], b.idx[f + 2], k, k, n, true, 0, step);
      collide_pair(pv, ld, m, b.dt, b.idx[f + 2], b.idx[f], k, k, n, true, 0, step);
      start = 3;
    }
    for (int a = start; a + 1 < N; a += 2)
      collide_pair(pv, ld, m, b.dt, b.idx[f + a], b.idx[f + a + 1], k, k, n, false, 0, step);
  }
  // unlike kinds
  for (int ga = 0; ga < G; ++ga) {
    const int ka = pick(gk, ga), fa = pick(gf, ga), Na = pick(gn, ga);
    const double ma = pick(mn13, ga);
    for (int gb = ga + 1; gb < G; ++gb) {
      const int kb = pick(gk, gb), fb = pick(gf, gb), Nb = pick(gn, gb);
      const int nmin = Na < Nb ? Na : Nb, nmax = Na < Nb ? Nb : Na;
      const double n = nmin * fmax(sw[ka], sw[kb]) / vcell, m = fmax(ma, pick(mn13, gb));
      for (int i = 0; i < nmax; ++i)
        collide_pair(pv, ld, m, b.dt, b.idx[fa + i % Na], b.idx[fb + i % Nb], ka, kb, n, false,
                     (uint32_t)(i / nmin), step);
    }
  }
  return true;
}

__global__ __launch_bounds__(CELLS_TPB, 2) void k_col_cells(const Inst I, ColBufs b, int step, int nb) {
  __shared__ double smass[MAXKIND], sw[MAXKIND];
  __shared__ uint64_t skey[SORT_LDS * CELLS_TPB];
  __shared__ int sidx[SORT_LDS * CELLS_TPB];
  if (threadIdx.x < MAXKIND) {
    smass[threadIdx.x] = I.kmass[threadIdx.x];
    sw[threadIdx.x] = I.kw[threadIdx.x];
  }
  __syncthreads();
  const PView pv{I.pu0, I.pu1, I.pu2, I.pid, I.seed, smass, sw};
  const ImpView iv{I.alive, I.death, I.no0, I.no1, I.no2, I.pcell, I.po0, I.po1, I.po2, I.pkind, I.pcount,
                   I.health, I.nevents, I.ksig, I.mat_cell, I.capacity, I.D, I.nx, I.ny, I.ppc};
  const int nact = b.bact[nb];
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < nact; q += gridDim.x * blockDim.x)
    collide_cell(b, pv, iv, I.pkind, I.vcell, smass, sw, skey + threadIdx.x, sidx + threadIdx.x, b.list[q], step);
}

}  // namespace

int col_scan_blocks(int n) { return (n + SCAN_B - 1) / SCAN_B; }

void launch_collide(const Inst& I, const ColBufs& b, int step, hipStream_t s, Stamp st) {
  const int n = b.ncell + 1;
  const int nb = col_scan_blocks(n);
  // grid-stride passes over the charged slots: one thread per slot up to 65536
  // blocks (each slot's loads and atomic are one dependent chain; more threads
  // keep more chains in flight)
  const int slots = 256 * std::min(65536, std::max(1, (I.capacity + 255) / 256));
  if (st.start)
    hipExtLaunchKernelGGL(k_col_clear, dim3((n + 255) / 256), dim3(256), 0, s, st.start, nullptr, 0, b);
  else
    hipLaunchKernelGGL(k_col_clear, dim3((n + 255) / 256), dim3(256), 0, s, b);
  hipLaunchKernelGGL(k_col_count, dim3(slots / 256), dim3(256), 0, s, I, b);
  hipLaunchKernelGGL(k_col_scan_local, dim3(nb), dim3(SCAN_B), 0, s, I, b, n);
  hipLaunchKernelGGL(k_col_scan_top, dim3(1), dim3(SCAN_B), 0, s, b, nb);
  hipLaunchKernelGGL(k_col_scan_add, dim3(nb), dim3(SCAN_B), 0, s, b, n);
  hipLaunchKernelGGL(k_col_fill, dim3(slots / 256), dim3(256), 0, s, I, b, step);
  // one thread per listed cell (at most one per slot), grid-stride
  const int cb = std::min(4096, std::max(1, (I.capacity + CELLS_TPB - 1) / CELLS_TPB));
  if (st.stop)
    hipExtLaunchKernelGGL(k_col_cells, dim3(cb), dim3(CELLS_TPB), 0, s, nullptr, st.stop, 0, I, b, step, nb);
  else
    hipLaunchKernelGGL(k_col_cells, dim3(cb), dim3(CELLS_TPB), 0, s, I, b, step, nb);
}

}  // namespace pic
