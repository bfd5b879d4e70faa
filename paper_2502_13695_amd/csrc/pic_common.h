// Shared definitions of the MI355X PIC library: the per-instance parameter
// block the kernels read, the Philox4x32-10 generator and the FP32 Keldysh
// table lookup (both usable on host and device).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

constexpr int G = 3;             // guard layers per side of every present axis
constexpr int MAXMAT = 8;
constexpr int MAXKIND = 2 * MAXMAT;
constexpr uint8_t DEAD = 0xFF;   // kind of an empty charged slot

// Health bits (latched in device memory, read by the diagnostics)
constexpr unsigned HEALTH_CAPACITY = 1u;
constexpr unsigned HEALTH_NONFINITE = 2u;

// Philox draw purposes (fourth counter word)
constexpr uint32_t PURPOSE_POS = 1, PURPOSE_VEL = 2, PURPOSE_IONIZE = 3,
                   PURPOSE_STRESS_E = 4, PURPOSE_STRESS_P = 5, PURPOSE_TRACK = 6;

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon et al., SC'11): counter (id_lo, id_hi, step, purpose),
// key (seed_lo, seed_hi).
struct u32x4 { uint32_t x, y, z, w; };

__host__ __device__ inline u32x4 philox4x32(u32x4 c, uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c = u32x4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
  }
  return c;
}

__host__ __device__ inline u32x4 draw(uint64_t seed, uint64_t id, uint32_t step, uint32_t purpose) {
  return philox4x32(u32x4{(uint32_t)id, (uint32_t)(id >> 32), step, purpose},
                    (uint32_t)seed, (uint32_t)(seed >> 32));
}

// Thermal velocity u = gamma v / c of a particle born from neutral `id`: three
// normal components of spread sig from one Philox block (counter (id, 0,
// purpose)).  Box-Muller in FP64, rounded once at the end: in FP32 the uniform
// next to 1 keeps only 24 bits of 1 - u, so -2 log u (hence a small radius)
// would carry relative errors up to 1e-3.
__device__ __forceinline__ void maxwell(uint64_t seed, uint64_t id, uint32_t purpose, float sig, float& ux,
                                         float& uy, float& uz) {
  const u32x4 w = draw(seed, id, 0u, purpose);
  const double u1 = ((double)w.x + 0.5) * 0x1p-32;
  const double u2 = ((double)w.y + 0.5) * 0x1p-32;
  const double u3 = ((double)w.z + 0.5) * 0x1p-32;
  const double u4 = ((double)w.w + 0.5) * 0x1p-32;
  const double r1 = sqrt(-2.0 * log(u1)), r2 = sqrt(-2.0 * log(u3));
  const double tp = 6.283185307179586476925;
  double s2, c2;
  sincos(tp * u2, &s2, &c2);
  const double sg = (double)sig;
  ux = (float)(sg * (r1 * c2));
  uy = (float)(sg * (r1 * s2));
  uz = (float)(sg * (r2 * cos(tp * u4)));
}

// ---------------------------------------------------------- Keldysh table
// Per material: P(A) = 1 - exp(-r(A)), r = W(A) dt / n0.  Between consecutive
// channel closings (x(A) crossing an integer, Eq. 1) the rate is
//   r(A) = S1(A) + sqrt(A_k - A) S2(A)
// with S1, S2 smooth: the n = 0 Dawson term of Eq. (3) vanishes like a square
// root at the closing A_k.  S1 and S2 are cubic polynomials in the local
// coordinate f = (A - A_i) / h of each interval of a uniform grid (step h)
// inside each segment.  Interval record: {A_i, S1 c0..c3, S2 c0..c3, pad x3}.
constexpr int TAB_REC = 12;

struct TabSeg {
  float lo, hi, inv_h;      // segment [lo, hi), 1 / grid step
  int base, nint;           // first interval, number of intervals
  int has_sigma;            // right end is a channel closing
  float dk;                 // exact closing A_k = hi - dk (0 <= dk < 1 ulp of hi)
  int pad1;
};

struct TabHdr {
  float acut;               // A < acut: P < 2^-34 (cannot fire against a u32 draw)
  float asat;               // A >= asat: P = 1
  int nseg;
  int pad;
};
// Memory: TabHdr, TabSeg[nseg], then float rec[TAB_REC * total intervals].

__host__ __device__ inline float table_lookup(const TabHdr* __restrict__ h, float A) {
  if (!(A >= h->acut)) return 0.0f;
  if (A >= h->asat) return 1.0f;
  const TabSeg* seg = reinterpret_cast<const TabSeg*>(h + 1);
  int k = 0;
  while (k + 1 < h->nseg && A >= seg[k].hi) ++k;
  const TabSeg s = seg[k];
  int i = (int)((A - s.lo) * s.inv_h);
  i = i < 0 ? 0 : (i >= s.nint ? s.nint - 1 : i);
  const float* c = reinterpret_cast<const float*>(seg + h->nseg) + TAB_REC * (s.base + i);
  const float f = (A - c[0]) * s.inv_h;
  float r = c[1] + f * (c[2] + f * (c[3] + f * c[4]));
  if (s.has_sigma) {
    const float s2 = c[5] + f * (c[6] + f * (c[7] + f * c[8]));
    const float d = (s.hi - A) - s.dk;   // A_k - A; hi - A is exact
    r += sqrtf(d > 0.0f ? d : 0.0f) * s2;
  }
  return -expm1f(-r);
}

// Upper bound of table_lookup(h, A') over every A' <= A (the records hold the
// running maximum of per-interval bounds, slot 9): a draw at or above it cannot
// fire for any amplitude up to A, so the amplitude itself need not be known.
// The same with the header fields and the segments from a copy (the records
// stay in the table at h).
__host__ __device__ inline float table_bound_at(const TabHdr* __restrict__ h, float acut, float asat, int nseg,
                                                const TabSeg* __restrict__ seg, float A) {
  if (!(A >= acut)) return 0.0f;
  if (A >= asat) return 1.0f;
  int k = 0;
  while (k + 1 < nseg && A >= seg[k].hi) ++k;
  const TabSeg s = seg[k];
  int i = (int)((A - s.lo) * s.inv_h);
  i = i < 0 ? 0 : (i >= s.nint ? s.nint - 1 : i);
  return reinterpret_cast<const float*>(reinterpret_cast<const TabSeg*>(h + 1) + nseg)[TAB_REC * (s.base + i) + 9];
}
__host__ __device__ inline float table_bound(const TabHdr* __restrict__ h, float A) {
  return table_bound_at(h, h->acut, h->asat, h->nseg, reinterpret_cast<const TabSeg*>(h + 1), A);
}

// ------------------------------------------------------ particle offsets
// A charged particle's offset in its cell is a 32-bit fraction o (t = o 2^-32,
// uniform resolution 2.3e-10 cells; an FP32 offset has 6e-8 near 1, which is
// 3e-5 of a thermal electron's step).  The shape weights take it as an FP32
// number; the Esirkepov differences and the move use the integer.
__host__ __device__ inline float off_lo(uint32_t o) {   // truncated to 24 bits, < 1
  return (float)(o >> 8) * 0x1p-24f;
}
__host__ __device__ inline float off_f32(uint32_t o) {  // nearest FP32 below 1
  const float t = (float)((double)o * 0x1p-32);
  return t < 1.0f ? t : 0x1.fffffep-1f;
}
__host__ __device__ inline uint32_t off_fix(float t) {   // t in [0, 1), exact for FP32 t
  return (uint32_t)((double)t * 0x1p32);
}

// ------------------------------------------------------- particle tiles
// The charged particles are kept sorted by tile of the deposit (counting sort,
// redone when enough particles have left their tile or landed beyond the
// layout).  A particle that starts a step in cell c deposits its current on
// nodes c - 2 .. c + 3 of each present axis (Esirkepov, shape order <= 2, at
// most one cell per step), so the deposit of a whole tile of T cells fits a
// window of T + 5 nodes held in LDS.  Each tile's range is followed by room
// for its births until the next sort: electrons and positive carriers in two
// halves, each as large as the tile's alive neutrals (immobile, ionized once).
__host__ __device__ constexpr int ptile_ext(int D, int axis) {
  return axis >= D ? 1 : (D == 1 ? 128 : (D == 2 ? 16 : (axis == 2 ? 4 : 8)));
}
__host__ __device__ constexpr int ptile_cells(int D) {
  return ptile_ext(D, 0) * ptile_ext(D, 1) * ptile_ext(D, 2);
}
constexpr int PT_LO = 2;            // window starts PT_LO nodes below the tile
constexpr int PT_PAD = 5;           // window = tile + PT_PAD nodes per present axis
// Ionization: a block of TPB threads takes TPB x ion_nit(ppc) consecutive
// neutrals (each thread up to ION_NIT of them), i.e. at most TPB cells.
constexpr int ION_NIT = 8;
constexpr int ION_SMAT = 2, ION_SSEG = 16;   // rate-table segments staged in LDS per block
__host__ __device__ constexpr int ion_nit(int64_t ppc) { return ppc < ION_NIT ? (int)ppc : ION_NIT; }
constexpr int SORT_CHUNK = 1024;    // sorted particles per work item (piece of a tile)
// Pieces of at most sparse_chunk(D) particles skip the LDS windows and add
// into HBM with FP32 atomics.  In 2D that is cheaper than staging and
// flushing a window for a handful of particles; in 3D the HBM atomics of a
// particle's three-dimensional stencil cost more than the window at any
// chunk size (measured on the mirror share and the pre-ionized stress run).
__host__ __device__ constexpr int sparse_chunk(int D) { return D == 3 ? 0 : 128; }
// LDS deposit in 64-bit fixed point: a contribution v (|v| <= max |kq|) is
// added as round(v * jscale) with jscale = 2^40 / 2^ceil(log2 max |kq|); a
// node's sum over one work item (the particles within two cells of it) stays
// far below 2^63; the sum is exact and does not depend on the order of the
// atomics.
constexpr int JFIX_BITS = 40;

// sort control words (device): [0] end of the layout (sorted tiles and their
// birth room), [1] chunks, [2] drifters deposited outside their tile's window
// since the sort (per step), [3] sort decision, [4] sorts performed, [5] a
// sort is wanted at the next check whatever the counts
constexpr int SC_NSORTED = 0, SC_NCHUNKS = 1, SC_NDRIFT = 2, SC_GO = 3, SC_NSORTS = 4, SC_FORCE = 5,
              SC_WORDS = 8;
// Charged region along x: cells [lo, hi] that held a charged particle at some
// step so far (never shrinks), in three rotating slots (step n reads slot n % 3,
// its push extends slot (n + 1) % 3).  Field tiles farther than XNEAR_MARGIN
// cells from it (and from the amplitude window) have carried no current, ever.
constexpr int XNEAR_MARGIN = 6;

// ----------------------------------------------------- instance parameters
struct Inst {
  // grid
  int D, order, nx, ny, nz;
  int Px, Py, Pz;               // padded extents (absent axes: 1)
  int sy, sz;                   // strides of y and z in the padded arrays
  int Gy, Gz;                   // guard offsets of y, z (0 if absent)
  int per_y, per_z;             // periodic transverse axes
  float C[3];                   // c dt / dx_d (FP32-exact)
  float halfC[3];
  float kmur[3];
  float ctdt_m;                 // c dt [m] (displacement along absent axes)
  // fields (padded, x fastest): F[parity][Ex, Ey, Ez, bx, by, bz]; the set
  // (step & 1) holds E^n, b^n; the field kernel writes the other set
  float* F[2][6];
  // current dt J / eps0: the push of step n deposits into Jb[n & 1]; the field
  // kernel of step n reads it and clears Jb[(n + 1) & 1] for the next push
  float* Jb[2][3];
  const float* ie_half;         // 1/eps_r at Ex positions, per padded x index
  const float* ie_node;         // 1/eps_r at nodes, per padded x index
  // Lorentz media: Q = P/eps0 (step n) and K = dt J_p/eps0 (step n - 1/2) in
  // set n & 1 at E positions, the field update writes set (n + 1) & 1; per
  // padded x the oscillator coefficients and the Kerr chi3 (a, c, c deps,
  // chi3) at Ex positions and at nodes.  Positions lx0 <= padded x < lx1 hold
  // every oscillator and Kerr term; null pointers and lx0 >= lx1 when the run
  // has none.
  float* Q[2][3];
  float* Kp[2][3];
  const float4* lor_half;
  const float4* lor_node;
  int lx0, lx1;
  const signed char* mat_cell;  // material of cell i (-1 vacuum), per cell x index
  // laser
  int pol;                      // 1 = Ey, 2 = Ez
  int nsrc;                     // entries in src
  const float4* src;            // per time level m: g(m dt), g(m dt - dx/c), 0, 0
  const float* prof;            // transverse profile of the polarised component (Py * Pz)
  // amplitude window (Sec. 2.1): node |E| over [wx0, wx1) padded x indices
  int nwin, wx0, wx1, wnx;      // wnx = wx1 - wx0
  int64_t wsz;                  // wnx * Py * Pz
  float *ring, *suffix, *prefix, *A;
  // charged particles (SoA)
  uint32_t* pcell;              // packed cell indices
  uint32_t *po0, *po1, *po2;     // offsets in the cell, 32-bit fractions (t = o 2^-32)
  float *pu0, *pu1, *pu2;
  uint8_t* pkind;
  uint32_t* pid;                // id of the parent neutral (placed particles: cells * ppc + index)
  int* pcount;                  // used slots
  int capacity;
  // tile sort: [0, sctl[SC_NSORTED]) holds the tiles in order, each range
  // followed by its birth room; particles placed or born beyond it follow up
  // to *pcount
  int ntile[3], ntiles;
  int* tcnt;                    // per tile: particles counted (zero between sorts)
  int* tstart;                  // first slot
  int* tbirth;                  // first birth slot (electrons; positive carriers tslack later)
  int* tslack;                  // birth room: events the tile can still take
  int* tfill;                   // events taken since the sort
  int* talive;                  // upper bound of the tile's alive neutrals
  int* tperm;                   // slot order inside the tile: rank r goes to (r tperm) mod count
  int4* chunks;                 // {tile, first slot, end slot, first birth slot or -1}
  float jscale, jscale_inv;     // LDS fixed-point scale of the deposit and its inverse
  int* sctl;                    // SC_* words
  uint32_t* scell;              // scatter targets (same layout as the particle arrays)
  uint32_t *so0, *so1, *so2;
  float *su0, *su1, *su2;
  uint8_t* skind;
  uint32_t* spid;
  // particle kinds: 2m electron, 2m+1 positive carrier
  float kh[MAXKIND];            // q dt / (2 m c)
  float kq[MAXKIND][3];         // qhat dx_d (present axes) or qhat c dt (absent)
  float ksig[MAXMAT];           // thermal velocity spread / c of the neutral molecules
  double kqhat[MAXKIND];        // q w / (eps0 V) [V/m^2] (diagnostics, FP64)
  double kw[MAXKIND];           // macroparticle weight (physical particles)
  double kmass[MAXKIND];        // mass [kg]
  double dx[3];                 // cell size [m] (absent axes: 1)
  double vcell;                 // cell volume [m^3] (absent axes count as 1 m)
  // neutrals
  int64_t nneut;
  int ppc;
  uint64_t ppc_magic;           // ceil(2^64 / ppc): neutral index / ppc by multiply-high
  float *no0, *no1, *no2;       // offsets
  uint32_t* alive;              // bitmask
  int* death;                   // ionization step, -1 alive
  const uint32_t* mcell;        // packed cell of each material cell (neutral / ppc)
  const TabHdr* tab[MAXMAT];
  int nmat;
  float acut[MAXMAT];
  float acut_min;               // smallest cut over the materials
  int* hot;                     // [step & 1]: some node's amplitude reached acut_min
  int* xext;                    // charged region, 3 slots x {lo, hi} (cells)
  int* front;                   // last padded x index of a tile that stored a nonzero E or b
  unsigned long long* tiles_done;   // field tiles updated, one counter per XCD (stride 32)
  unsigned long long* nevents;  // per XCD and material: [x * 32 + m]
  int* pq;                      // push work queues: next item of XCD x's range at [64 x], blocks done at [512]
  // field energy through the flux surface (the faces of the box one cell
  // inside the outflow faces), J, per XCD x: [x * 32] entering, [x * 32 + 1]
  // leaving
  double* eflux;
  double kflux[3];              // eps0 c dt x the transverse cell area of a plane normal to axis d
  uint64_t seed;
  // control
  int* step;                    // device step counter
  int step_now;                 // batches: the step index, kept by k_advance beside the counter
  unsigned* health;
};

// packed cell: D = 1: i; D = 2: i | j << 16; D = 3: i | j << 12 | k << 22
__host__ __device__ inline uint32_t pack_cell(int D, int i, int j, int k) {
  if (D == 1) return (uint32_t)i;
  if (D == 2) return (uint32_t)i | ((uint32_t)j << 16);
  return (uint32_t)i | ((uint32_t)j << 12) | ((uint32_t)k << 22);
}
__host__ __device__ inline void unpack_cell(int D, uint32_t c, int& i, int& j, int& k) {
  if (D == 1) { i = (int)c; j = 0; k = 0; return; }
  if (D == 2) { i = (int)(c & 0xFFFFu); j = (int)(c >> 16); k = 0; return; }
  i = (int)(c & 0xFFFu); j = (int)((c >> 12) & 0x3FFu); k = (int)(c >> 22);
}

}  // namespace pic
