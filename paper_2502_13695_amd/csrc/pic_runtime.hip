// C ABI of the MI355X PIC library (include/pic.h): context set-up, device
// memory layout, stepping, batching and diagnostics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "host_math.h"
#include "pic.h"
#include "pic_kernels.h"

using namespace pic;

namespace {

constexpr double kC = 299792458.0;
constexpr double kQE = 1.602176634e-19;
constexpr double kEPS0 = 8.8541878128e-12;
constexpr double kKB = 1.380649e-23;

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Process-wide cache of the FP64-built rate tables: a table depends only on
// the material, the wavelength, the time step and the number of terms, which
// runs of a scan or a serving mix share (building one takes ~0.4 s of host time).
pic_status cached_table(const Canon& c, int mat, int terms, int tol_bits, TableHost* out) {
  static std::mutex mu;
  static std::map<std::string, TableHost> cache;
  const MatC& m = c.mats[mat];
  const double key_v[9] = {m.gap_eV, m.n_index, m.n0, m.mred, m.mol_kg, m.e_kg, m.p_kg, c.lam, c.dt};
  std::string key(reinterpret_cast<const char*>(key_v), sizeof key_v);
  key.append(reinterpret_cast<const char*>(&terms), sizeof terms);
  key.append(reinterpret_cast<const char*>(&tol_bits), sizeof tol_bits);
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(key);
    if (it != cache.end()) {
      *out = it->second;
      return PIC_OK;
    }
  }
  const pic_status st = build_table(c, mat, terms, out, tol_bits);
  if (st != PIC_OK) return st;
  std::lock_guard<std::mutex> g(mu);
  if (cache.size() >= 256) cache.clear();
  cache.emplace(key, *out);
  return PIC_OK;
}

// Device memory plan of one context (offsets into one allocation).
struct Layout {
  int64_t Px, Py, Pz, ncell;
  int64_t nmcell, nneut, capacity;
  int wx0, wx1;
  int64_t wsz;
  int nsrc;
  size_t o_F[2][6], o_J[2][3], o_ie_half, o_ie_node, o_mat, o_src, o_prof;
  // Lorentz media: polarisation Q and its current K (two sets, as the fields),
  // per-x oscillator coefficients; lx0 <= padded x < lx1 spans every position
  // with an oscillator (lx0 >= lx1: none, nothing allocated)
  size_t o_Q[2][3], o_Kp[2][3], o_lor_half, o_lor_node;
  int lx0, lx1;
  bool kerr = false;   // some Kerr term inside [lx0, lx1)
  // binary collisions: per-cell counts and starts, fill counters, scan block
  // sums, slots ordered by cell and their pairing keys (empty without collisions)
  size_t o_ccnt, o_cfill, o_cbsum, o_cidx, o_ckey, o_cact, o_mrank;
  size_t o_ring, o_suffix, o_prefix, o_A;
  size_t o_no[3], o_alive, o_death, o_mcell;
  size_t o_pcell, o_po[3], o_pu[3], o_pkind, o_pid;
  int ntile[3];
  int64_t ntiles, maxchunks;
  size_t o_tcnt, o_tstart, o_tbirth, o_tslack, o_tfill, o_talive, o_tperm, o_chunks;
  size_t o_scell, o_so[3], o_su[3], o_skind, o_spid;
  size_t o_tab[MAXMAT];
  size_t o_ctr;      // pcount, step, health, nevents[MAXMAT], diag accumulators
  size_t o_grid64;   // FP64 node grid for diagnostics
  size_t o_inst, o_off, o_sig;
  size_t o_probe;    // scratch for table probes
  size_t total;
};

// the field update's dispersive variant of a layout (Group::lor)
static int disp_mode(const Layout& L) { return L.lx0 < L.lx1 ? (L.kerr ? 2 : 1) : 0; }

// Device counters.  Words that every block of a launch reads (the step of a
// batch member, the charged region) sit on cache lines of their own, apart
// from the words that blocks update with atomics while others read.
struct Ctr {
  alignas(256) int step;
  alignas(256) int xext[6];
  alignas(256) int front;
  alignas(256) unsigned long long tiles_done[8 * 32];   // one 256-byte line per XCD
  alignas(256) int pcount;
  unsigned health;
  unsigned done;
  alignas(256) int sctl[SC_WORDS];
  alignas(256) int hot[2];
  // counts added from every block: one 256-byte line per XCD (slot x * 32 + m),
  // summed when read; same-address atomics from all XCDs serialize
  alignas(256) unsigned long long nevents[8 * 32];
  double acc[64];
  alignas(256) int pq[9 * 64];   // push work queues (one 256-byte line each), zero between launches
  alignas(256) double eflux[8 * 32];   // into / out of the flux surface [J]: slots x * 32 + 0 / 1
};

pic_status plan(const pic_config* cfg, const Canon& c, const std::vector<TableHost>& tabs, Layout* L) {
  const int D = c.D;
  L->Px = c.n[0] + 1 + 2 * G;
  L->Py = D >= 2 ? c.n[1] + 1 + 2 * G : 1;
  L->Pz = D >= 3 ? c.n[2] + 1 + 2 * G : 1;
  L->ncell = L->Px * L->Py * L->Pz;
  int64_t nxm = 0, imin = -1, imax = -1;
  for (int64_t i = 0; i < c.n[0]; ++i)
    if (c.mat_cell[i] >= 0) {
      ++nxm;
      if (imin < 0) imin = i;
      imax = i;
    }
  L->nmcell = nxm * c.n[1] * c.n[2];
  L->nneut = L->nmcell * c.ppc;
  if (nxm > 0) {
    L->wx0 = (int)std::max<int64_t>(0, imin - 1) + G;
    L->wx1 = (int)std::min<int64_t>(c.n[0], imax + 2) + G + 1;
  } else {
    L->wx0 = L->wx1 = G;
  }
  L->wsz = (int64_t)(L->wx1 - L->wx0) * L->Py * L->Pz;
  int64_t cap = cfg->particle_capacity > 0 ? cfg->particle_capacity : 2 * L->nneut + 4096;
  if (cfg->preionize_eV > 0) cap = std::max<int64_t>(cap, 2 * L->nneut);
  // particle tiles
  L->ntiles = 1;
  for (int d = 0; d < 3; ++d) {
    const int64_t e = ptile_ext(D, d);
    L->ntile[d] = d < D ? (int)((c.n[d] + e - 1) / e) : 1;
    L->ntiles *= L->ntile[d];
  }
  // grid byte offsets are 32-bit in the kernels
  if (cap > INT_MAX / 2 || L->ntiles > (1 << 26) || L->nneut > ((int64_t)1 << 40) || c.ppc > 65535 ||
      L->ncell >= (1 << 30))
    return PIC_E_INVAL;
  L->capacity = cap;
  // chunks: ceil(n / SORT_CHUNK) per tile with particles, one per tile with
  // birth room only
  L->maxchunks = 2 * L->ntiles + cap / SORT_CHUNK + 1;
  // source samples cover the planned steps and the whole pulse (Gaussian: to
  // t0 + 8 fwhm, where the envelope is below 1e-38; sin^2: its full length)
  const double t_end = c.env == PIC_ENV_GAUSS ? c.t0 + 8.0 * c.fwhm : c.t0 + 0.5 * c.T;
  const int64_t pulse_steps = (int64_t)std::ceil(t_end / c.dt) + 2;
  L->nsrc = (int)std::min<int64_t>(std::max<int64_t>(cfg->nsteps + 2, pulse_steps), 1 << 26);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o += align256(bytes);
    return r;
  };
  const size_t f = sizeof(float) * (size_t)L->ncell;
  for (int par = 0; par < 2; ++par)
    for (int q = 0; q < 6; ++q) L->o_F[par][q] = take(f);
  for (int par = 0; par < 2; ++par)
    for (int q = 0; q < 3; ++q) L->o_J[par][q] = take(f);
  L->o_ie_half = take(sizeof(float) * L->Px);
  L->o_ie_node = take(sizeof(float) * L->Px);
  L->lx0 = (int)L->Px;
  L->lx1 = 0;
  for (int64_t i = 0; i <= c.n[0]; ++i) {
    // Lorentz oscillators or a Kerr term (both in the field update's dispersive variant)
    auto disp = [&](int m) { return m >= 0 && (c.mats[m].lam0 > 0 || c.mats[m].chi3 != 0.0f); };
    const bool lc = i < c.n[0] && disp(c.mat_cell[i]);
    const bool ln = disp(c.mat_node[i]);
    if (lc || ln) {
      L->lx0 = std::min(L->lx0, (int)(i + G));
      L->lx1 = std::max(L->lx1, (int)(i + G + 1));
    }
    auto kerr = [&](int m) { return m >= 0 && c.mats[m].chi3 != 0.0f; };
    if ((i < c.n[0] && kerr(c.mat_cell[i])) || kerr(c.mat_node[i])) L->kerr = true;
  }
  const size_t fq = L->lx0 < L->lx1 ? f : 0;
  for (int par = 0; par < 2; ++par)
    for (int q = 0; q < 3; ++q) {
      L->o_Q[par][q] = take(fq);
      L->o_Kp[par][q] = take(fq);
    }
  L->o_lor_half = take(fq ? sizeof(float4) * L->Px : 0);
  L->o_lor_node = take(fq ? sizeof(float4) * L->Px : 0);
  L->o_mat = take(c.n[0]);
  L->o_src = take(sizeof(float) * 4 * (size_t)L->nsrc);
  L->o_prof = take(sizeof(float) * L->Py * L->Pz);
  L->o_ring = take(sizeof(float) * (size_t)L->wsz * c.nwin);
  L->o_suffix = take(sizeof(float) * (size_t)L->wsz * c.nwin);
  L->o_prefix = take(sizeof(float) * (size_t)L->wsz);
  L->o_A = take(f);
  for (int q = 0; q < 3; ++q) L->o_no[q] = take(q < D ? sizeof(float) * L->nneut : 0);
  L->o_alive = take(sizeof(uint32_t) * ((L->nneut + 31) / 32 + 1));
  L->o_death = take(sizeof(int) * L->nneut);
  L->o_mcell = take(sizeof(uint32_t) * L->nmcell);
  L->o_pcell = take(sizeof(uint32_t) * L->capacity);
  for (int q = 0; q < 3; ++q) L->o_po[q] = take(q < D ? sizeof(uint32_t) * L->capacity : 0);
  for (int q = 0; q < 3; ++q) L->o_pu[q] = take(sizeof(float) * L->capacity);
  L->o_pkind = take(L->capacity);
  L->o_pid = take(sizeof(uint32_t) * L->capacity);
  L->o_tcnt = take(sizeof(int) * L->ntiles);
  L->o_tstart = take(sizeof(int) * L->ntiles);
  L->o_tbirth = take(sizeof(int) * L->ntiles);
  L->o_tslack = take(sizeof(int) * L->ntiles);
  L->o_tfill = take(sizeof(int) * L->ntiles);
  L->o_talive = take(sizeof(int) * L->ntiles);
  L->o_tperm = take(sizeof(int) * L->ntiles);
  L->o_chunks = take(sizeof(int4) * L->maxchunks);
  L->o_scell = take(sizeof(uint32_t) * L->capacity);
  for (int q = 0; q < 3; ++q) L->o_so[q] = take(q < D ? sizeof(uint32_t) * L->capacity : 0);
  for (int q = 0; q < 3; ++q) L->o_su[q] = take(sizeof(float) * L->capacity);
  L->o_skind = take(L->capacity);
  L->o_spid = take(sizeof(uint32_t) * L->capacity);
  for (int m = 0; m < MAXMAT; ++m) L->o_tab[m] = take(m < (int)tabs.size() ? tabs[m].bytes.size() : 0);
  L->o_ctr = take(sizeof(Ctr));
  L->o_grid64 = take(sizeof(double) * (size_t)L->ncell);
  L->o_inst = take(sizeof(Inst));
  L->o_off = take(sizeof(int) * 32);   // 4 phases x {0, blocks}; field shapes x {0, blocks}; the sort
  L->o_sig = take(sizeof(float) * 2 * MAXMAT);
  L->o_probe = take(0);
  {
    // binary collisions and impact ionization share the per-step cell binning
    const bool on = c.collide || c.impact;
    const int64_t nbox = on ? c.n[0] * c.n[1] * c.n[2] : 0;
    if (nbox >= (int64_t)1 << 30) return PIC_E_INVAL;   // cell indices and their scan are int
    const int64_t cap = on ? L->capacity : 0;
    L->o_ccnt = take(sizeof(int) * (size_t)(nbox + 1));
    L->o_cfill = take(sizeof(int) * (size_t)nbox);
    L->o_cbsum = take(sizeof(int) * (size_t)(on ? col_scan_blocks((int)nbox + 1) + 1 : 0));
    L->o_cidx = take(sizeof(int) * (size_t)cap);
    L->o_ckey = take(sizeof(uint64_t) * (size_t)cap);
    // listed cells per scan block, the blocks' counts and their total, the list
    L->o_cact = take(sizeof(int) * (size_t)(on ? (int64_t)col_scan_blocks((int)nbox + 1) * (COL_SCAN_B + 1) + 1 + cap
                                               : 0));
    L->o_mrank = take(sizeof(int) * (size_t)(on ? c.n[0] : 0));
  }
  L->total = o;
  return PIC_OK;
}

}  // namespace

struct pic_ctx {
  pic_config cfg{};
  std::vector<pic_material> mats;
  std::vector<pic_layer> layers;
  Canon canon;
  std::vector<TableHost> tabs;
  Layout L{};
  unsigned char* base = nullptr;
  hipStream_t stream = nullptr;
  Inst h{};
  Inst* d_inst = nullptr;
  ColBufs col{};   // binary collisions (when the run has them)
  int* d_off = nullptr;   // [0, nb_push, 0, nb_cell, 0, 1, 0, nb_neut], then {0, tiles} per field shape
  int* d_off_fields = nullptr;   // block offsets of the field launch in use
  int nb_push = 0, nb_cell = 0, nb_win = 0, nb_neut = 0, nb_sort = 0;
  int tile = 0;               // field-kernel tile variant
  double tune_ms[8] = {0};    // autotuner: ms per field launch of each variant
  // in-run tuning of the field tile shape: the next tune_left steps cycle the
  // shapes (tune_reps steps each; results identical), timing every launch
  int tune_left = 0, tune_reps = 0;
  int nvar = 7;                // field tile shapes this run can use
  hipEvent_t tune_ev[8][16][2] = {};
  Ctr* d_ctr = nullptr;
  double* d_grid64 = nullptr;
  std::vector<uint32_t> mcell;
  int64_t step = 0;
  pic_status latched = PIC_OK;
  int timing = 0;             // 0 off; k > 0: time the launches of every k-th step
  double timers[8] = {0};     // accumulated ms per phase
  double tcount[8] = {0};     // launches timed per phase
  // event ring per phase: record around each launch, read back when reused
  static constexpr int kRing = 64;
  hipEvent_t ev[8][kRing][2] = {};
  int ev_used[8][kRing] = {};
  int64_t ev_slot = 0;
  int owns_alloc_via_cb = 0;
  int* h_step = nullptr;      // pinned: staging for the device step counter
  int resort = 8;             // tile-sort check every `resort` steps (0 = never)
  int far_skip = 1;           // far field tiles skip the current (pic_set_far_tiles)
  int h_xext[6] = {};         // host source of the charged-region slots
  int imax_every = 0;         // node |E|^2 maximum sampled every k steps (0 off)
  float* d_imax = nullptr;    // its running maximum (padded grid), allocated on demand
  void* d_spec = nullptr;     // energy histogram: edges and counts, allocated on demand
  int track_every = 0;        // trajectory records every k steps (0 off)
  uint32_t track_thr = 0;     // sampled iff the id's Philox word is below this
  int64_t track_max = 0;      // records kept
  void* d_tracks = nullptr;   // record counter (256 B), then the records
};

struct pic_batch {
  std::vector<pic_ctx*> members;
  bool dirty = true;
  // per (D, order) class: device Inst copies and per-phase block offsets
  struct Class {
    int D, order, tile = 0;
    bool per = false;   // periodic transverse axes
    int lor = 0;        // dispersive variant: the largest of the members' (Group::lor)
    std::vector<pic_ctx*> ms;
    Inst* d_insts = nullptr;
    int* d_off = nullptr;   // 4 phases x (n + 1)
    unsigned short* d_map = nullptr;   // per phase: member of every block
    int map_off[4] = {0, 0, 0, 0};
    int n = 0;
    int blocks[4] = {0, 0, 0, 0};
  };
  std::vector<Class> classes;
  hipStream_t stream = nullptr;
  int resort = 8;     // tile-sort check every `resort` batch steps (0 = never)
  int64_t tick = 0;   // batch steps taken
  // one sort period of batch steps captured as a HIP graph (recaptured after
  // every change of membership), replayed on `stream`
  int graph_on = 1;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t replays = 0;
  std::vector<int64_t> expect;   // each member's step index as the batch's blocks hold it
};

namespace {

#define HIP_OK(x)                                   \
  do {                                              \
    if ((x) != hipSuccess) return PIC_E_DEVICE;     \
  } while (0)

inline void* devp(pic_ctx* c, size_t off) { return c->base + off; }

// first id of particles placed by pic_set_state: cells x ppc (every neutral
// id, cell index x ppc + k, lies below it)
int64_t placed_id_base(const pic_ctx* c) {
  int64_t cells = 1;
  for (int d = 0; d < c->canon.D; ++d) cells *= c->canon.n[d];
  return cells * (c->canon.ppc > 0 ? c->canon.ppc : 1);
}

// device memory beyond the state block, from the caller's allocator when given
void* dev_alloc(pic_ctx* c, size_t bytes) {
  if (c->cfg.alloc) return c->cfg.alloc(bytes, c->cfg.alloc_user);
  void* p = nullptr;
  return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
}
void dev_free(pic_ctx* c, void* p) {
  if (!p) return;
  if (c->cfg.alloc) {
    if (c->cfg.free) c->cfg.free(p, c->cfg.alloc_user);
  } else {
    (void)hipFree(p);
  }
}

// Energy histogram buffer: up to kSpecEdges edges, then MAXKIND rows of counts.
constexpr int kSpecEdges = 4097;
constexpr size_t kSpecBytes = sizeof(double) * kSpecEdges + sizeof(unsigned long long) * MAXKIND * (kSpecEdges + 1);

// Staging of the allocation-free energy histogram (pic_spectrum_counts_noalloc):
// the edges and counts of one call, up to the same maximum as the allocating
// entry point (557 KB).  Every GPU the library runs on holds one copy until the
// process ends; calls on one GPU share it.
static __device__ __align__(256) unsigned char scratch[kSpecBytes];

// Its device address on each GPU, resolved with that GPU current (pic_init,
// or the entry point's first call on a GPU no context was created on).
constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

pic_status scratch_ptr(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PIC_E_DEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PIC_E_DEVICE;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return PIC_OK;
}

// offsets of the tile sort's grid in the block-offset table (after the
// field shapes' pairs at 8 ..)
constexpr int PH_SORT = 12;
static_assert(2 * PH_SORT + 1 < 32, "block-offset table");

Group single(pic_ctx* c, int phase, int nb) {
  Group g{c->d_inst, phase == 1 ? c->d_off_fields : c->d_off + 2 * phase, 1, nb, (int)c->step};
  g.front = &c->d_ctr->front;
  g.xext = c->d_ctr->xext;
  g.host = &c->h;
  g.lor = disp_mode(c->L);
  return g;
}

// Timing events: no system-scope fence when they complete, so stamping a
// launch adds no cache write-back and invalidation around it.
hipError_t timing_event(hipEvent_t* e) { return hipEventCreateWithFlags(e, hipEventDisableSystemFence); }

// Phase timing: events stamped by the phase's dispatches on the context stream;
// a ring slot is read back (and accumulated) before it is reused.
void harvest(pic_ctx* c, int ph, int slot) {
  if (!c->ev_used[ph][slot]) return;
  float ms = 0.f;
  if (hipEventSynchronize(c->ev[ph][slot][1]) == hipSuccess &&
      hipEventElapsedTime(&ms, c->ev[ph][slot][0], c->ev[ph][slot][1]) == hipSuccess) {
    c->timers[ph] += ms;
    c->tcount[ph] += 1.0;
  }
  c->ev_used[ph][slot] = 0;
}

// one step in every window of `timing` steps, at an offset that advances by one
// per window (every residue of the step index is sampled equally often)
bool sampled(const pic_ctx* c) {
  return c->timing && c->step % c->timing == (c->step / c->timing) % c->timing;
}

// the node |E|^2 maximum after the field update of the current step (its new
// E is the parity the update wrote)
ImaxArgs imax_args(const pic_ctx* c) {
  const Inst& I = c->h;
  const int np = (int)((c->step & 1) ^ 1);
  ImaxArgs a{};
  a.E0 = I.F[np][0];
  a.E1 = I.F[np][1];
  a.E2 = I.F[np][2];
  a.D = I.D;
  a.nx = I.nx;
  a.ny = I.ny;
  a.nz = I.nz;
  a.per_y = I.per_y;
  a.per_z = I.per_z;
  a.Gy = I.Gy;
  a.Gz = I.Gz;
  a.sy = I.sy;
  a.sz = I.sz;
  a.mx = I.nx + 1;
  a.my = I.D >= 2 ? (I.per_y ? I.ny : I.ny + 1) : 1;
  const int mz = I.D >= 3 ? (I.per_z ? I.nz : I.nz + 1) : 1;
  a.nodes = (int64_t)a.mx * a.my * mz;
  return a;
}

template <typename F>
void timed(pic_ctx* c, int ph, F&& launch) {
  if (!sampled(c)) {
    launch(Stamp{});
    return;
  }
  const int slot = (int)(c->ev_slot % pic_ctx::kRing);
  harvest(c, ph, slot);
  if (!c->ev[ph][slot][0]) {
    if (timing_event(&c->ev[ph][slot][0]) != hipSuccess || timing_event(&c->ev[ph][slot][1]) != hipSuccess) {
      launch(Stamp{});
      return;
    }
  }
  launch(Stamp{c->ev[ph][slot][0], c->ev[ph][slot][1]});
  c->ev_used[ph][slot] = 1;
}

// Charged region of every slot: cells [lo, hi] (with the amplitude window's
// cells); lo > hi = empty.
void set_region(pic_ctx* c, int lo, int hi) {
  const Layout& L = c->L;
  if (L.wx1 > L.wx0) {
    lo = std::min(lo, L.wx0 - G);
    hi = std::max(hi, L.wx1 - 1 - G);
  }
  for (int k = 0; k < 3; ++k) {
    c->h_xext[2 * k] = lo;
    c->h_xext[2 * k + 1] = hi;
  }
}

void harvest_all(pic_ctx* c) {
  for (int ph = 0; ph < 8; ++ph)
    for (int k = 0; k < pic_ctx::kRing; ++k) harvest(c, ph, k);
}

// phases: 0 push, 1 fields (Yee step, outflow faces, amplitude window),
// 2 ionize (+ step counter), 3 tile sort (when a check is due)
// End of the in-run tuning: the fastest shape (best of its launches) is kept.
void finish_tuning(pic_ctx* c) {
  const int nv = c->nvar;
  (void)hipEventSynchronize(c->tune_ev[nv - 1][c->tune_reps - 1][1]);
  double best = 1e30;
  for (int v = 0; v < nv; ++v) {
    c->tune_ms[v] = 1e30;
    for (int r = 0; r < c->tune_reps; ++r) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, c->tune_ev[v][r][0], c->tune_ev[v][r][1]) == hipSuccess)
        c->tune_ms[v] = std::min(c->tune_ms[v], (double)ms);
    }
    if (c->tune_ms[v] < best) {
      best = c->tune_ms[v];
      c->tile = v;
    }
  }
  const Layout& L = c->L;
  c->nb_cell = field_tiles(c->canon.D, c->tile, (int)L.Px, (int)L.Py, (int)L.Pz);
  c->d_off_fields = c->d_off + 8 + 2 * c->tile;
}

// The step's field update completes a block of amplitude-window samples
// (slot nwin - 1): the suffix maxima are rebuilt after it.
static bool rebuild_due(const pic_ctx* c) {
  const int nwin = c->canon.nwin;
  return nwin > 0 && c->L.wsz > 0 && c->step % nwin == nwin - 1;
}

void enqueue_step(pic_ctx* c) {
  const int D = c->canon.D, order = c->cfg.shape_order;
  hipStream_t s = c->stream;
  if (c->resort > 0 && c->step % c->resort == 0)
    timed(c, 3, [&](Stamp st) { launch_sort(single(c, PH_SORT, c->nb_sort), single(c, 2, 1), D, s, st); });
  timed(c, 0, [&](Stamp st) { launch_push(single(c, 0, c->nb_push), D, order, c->canon.per[1], s, st); });
  if (c->tune_left > 0) {
    const int idx = c->nvar * c->tune_reps - c->tune_left;
    const int v = idx / c->tune_reps, r = idx % c->tune_reps;
    const Layout& L = c->L;
    // every tile is updated while the shapes are timed (with tiles beyond the
    // field front skipped, the first steps would time an unrepresentative load)
    Group gv{c->d_inst, c->d_off + 8 + 2 * v, 1, field_tiles(D, v, (int)L.Px, (int)L.Py, (int)L.Pz),
             (int)c->step, c->far_skip ? 2 : 0};
    gv.front = &c->d_ctr->front;
    gv.xext = c->d_ctr->xext;
    gv.host = &c->h;
    gv.lor = disp_mode(c->L);
    launch_fields(gv, D, v, s, Stamp{c->tune_ev[v][r][0], c->tune_ev[v][r][1]});
    if (rebuild_due(c)) launch_win_rebuild(c->h, c->L.wsz, s);
    if (--c->tune_left == 0) finish_tuning(c);
  } else {
    timed(c, 1, [&](Stamp st) {
      Group g = single(c, 1, c->nb_cell);
      g.part = c->far_skip;
      // the window's suffix rebuild, when due, belongs to the field phase
      const bool rb = rebuild_due(c);
      launch_fields(g, D, c->tile, s, rb ? Stamp{st.start, nullptr} : st);
      if (rb) launch_win_rebuild(c->h, c->L.wsz, s, st.stop);
    });
  }
  if (c->imax_every > 0 && (c->step + 1) % c->imax_every == 0) launch_imax(imax_args(c), c->d_imax, s);
  timed(c, 2, [&](Stamp st) { launch_ionize(single(c, 3, c->nb_neut), D, order, s, st); });
  if (c->canon.collide || c->canon.impact)
    timed(c, 4, [&](Stamp st) { launch_collide(c->h, c->col, (int)(c->step + 1), s, st); });
  if (c->track_every > 0 && (c->step + 1) % c->track_every == 0)
    launch_tracks(c->d_inst, D, (int)c->L.capacity, c->track_thr, (int)(c->step + 1),
                  (TrackRec*)((unsigned char*)c->d_tracks + 256), (unsigned long long*)c->d_tracks,
                  c->track_max, s);
  if (sampled(c)) ++c->ev_slot;
  ++c->step;
}

// tile-sort grid: grid-stride blocks sized by the slot capacity, 8 slots per
// thread, 16 .. 2048, a multiple of 8 (the XCD count)
int sort_blocks(int64_t capacity) {
  const int64_t nb = (capacity + TPB * 8 - 1) / (TPB * 8);
  return (int)((std::max<int64_t>(16, std::min<int64_t>(nb, 2048)) + 7) / 8 * 8);
}

// padded index of logical (i, j, k)
inline int64_t pidx(const Layout& L, int D, int64_t i, int64_t j, int64_t k) {
  return (i + G) + L.Px * ((D >= 2 ? j + G : 0) + L.Py * (D >= 3 ? k + G : 0));
}

// domain extent of a component along axis d (half: staggered by 1/2)
inline int64_t dom_n(const Canon& c, int d, bool half) {
  if (d >= c.D) return 1;
  return (half || c.per[d]) ? c.n[d] : c.n[d] + 1;
}

template <typename Fn>
void for_domain(const Canon& c, const bool half[3], Fn fn) {
  const int64_t nx = dom_n(c, 0, half[0]), ny = dom_n(c, 1, half[1]), nz = dom_n(c, 2, half[2]);
  int64_t q = 0;
  for (int64_t k = 0; k < nz; ++k)
    for (int64_t j = 0; j < ny; ++j)
      for (int64_t i = 0; i < nx; ++i) fn(q++, i, j, k);
}

const bool kHalfE[3][3] = {{true, false, false}, {false, true, false}, {false, false, true}};
const bool kHalfB[3][3] = {{false, true, true}, {true, false, true}, {true, true, false}};
const bool kNode[3] = {false, false, false};

int64_t dom_count(const Canon& c, const bool half[3]) {
  return dom_n(c, 0, half[0]) * dom_n(c, 1, half[1]) * dom_n(c, 2, half[2]);
}

pic_status check_health(pic_ctx* c) {
  unsigned h = 0;
  HIP_OK(hipMemcpy(&h, &c->d_ctr->health, sizeof h, hipMemcpyDeviceToHost));
  if (c->latched == PIC_OK) {
    if (h & HEALTH_NONFINITE) c->latched = PIC_E_NUMERIC;
    else if (h & HEALTH_CAPACITY) c->latched = PIC_E_CAPACITY;
  }
  return PIC_OK;
}

// Arguments of an energy-histogram call.
pic_status spectrum_check(pic_ctx* c, const pic_spectrum* sp, const uint64_t* out, size_t out_count) {
  if (!c || !sp || !out) return PIC_E_INVAL;
  const int ne = sp->nedges;
  const int nk = 2 * c->canon.nmat;
  if (ne < 2 || ne > kSpecEdges || !sp->edges_eV) return PIC_E_INVAL;
  if (out_count != (size_t)nk * (size_t)(ne + 1)) return PIC_E_INVAL;
  for (int q = 0; q < ne; ++q) {
    if (!std::isfinite(sp->edges_eV[q])) return PIC_E_INVAL;
    if (q > 0 && !(sp->edges_eV[q] > sp->edges_eV[q - 1])) return PIC_E_INVAL;
  }
  if (sp->x_hi_cell > sp->x_lo_cell && (sp->x_lo_cell < INT32_MIN || sp->x_hi_cell > INT32_MAX)) return PIC_E_INVAL;
  return PIC_OK;
}

// The histogram through a device buffer of kSpecBytes (edges, then counts).
pic_status spectrum_into(pic_ctx* c, const pic_spectrum* sp, uint64_t* out, size_t out_count, void* buf) {
  hipStream_t s = c->stream;
  if (hipStreamSynchronize(s) != hipSuccess) return PIC_E_DEVICE;
  check_health(c);
  const int ne = sp->nedges;
  const int nk = 2 * c->canon.nmat;
  double* d_edges = (double*)buf;
  unsigned long long* d_cnt = (unsigned long long*)(d_edges + kSpecEdges);
  SpecArgs a{};
  a.nkinds = nk;
  a.nedges = ne;
  a.x_lo = sp->x_hi_cell > sp->x_lo_cell ? (int)sp->x_lo_cell : 0;
  a.x_hi = sp->x_hi_cell > sp->x_lo_cell ? (int)sp->x_hi_cell : 0;
  a.lds = (int)spec_lds_counts(nk, ne);
  // rest energy per kind [eV]: m c^2 / e
  for (int k = 0; k < nk; ++k) a.mc2_eV[k] = c->h.kmass[k] * kC * kC / kQE;
  HIP_OK(hipMemcpyAsync(d_edges, sp->edges_eV, sizeof(double) * ne, hipMemcpyHostToDevice, s));
  HIP_OK(hipMemsetAsync(d_cnt, 0, sizeof(unsigned long long) * out_count, s));
  launch_spectrum(c->d_inst, c->canon.D, (int)c->L.capacity, a, d_edges, d_cnt, s);
  HIP_OK(hipGetLastError());
  HIP_OK(hipMemcpyAsync(out, d_cnt, sizeof(unsigned long long) * out_count, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  return PIC_OK;
}

}  // namespace

extern "C" {

const char* pic_status_str(pic_status s) {
  switch (s) {
    case PIC_OK: return "ok";
    case PIC_E_INVAL: return "invalid argument";
    case PIC_E_NOMEM: return "device allocation failed";
    case PIC_E_DEVICE: return "HIP runtime error";
    case PIC_E_STATE: return "invalid state (latched error)";
    case PIC_E_NUMERIC: return "non-finite value";
    case PIC_E_CAPACITY: return "charged-particle capacity exceeded";
    case PIC_E_VERSION: return "ABI version mismatch";
  }
  return "unknown";
}

pic_status pic_canonical(const pic_config* cfg, pic_params* out) {
  if (!cfg || !out) return PIC_E_INVAL;
  Canon c;
  pic_status st = canonicalize(cfg, &c);
  if (st != PIC_OK) return st;
  std::memset(out, 0, sizeof *out);
  out->dt = c.dt;
  for (int d = 0; d < 3; ++d) {
    out->Cd[d] = c.C[d];
    out->kmur[d] = c.kmur[d];
  }
  for (int m = 0; m < c.nmat; ++m) {
    out->ie[m] = c.mats[m].ie;
    for (int q = 0; q < 3; ++q) out->lor[m][q] = c.mats[m].lor[q];
    out->chi3[m] = c.mats[m].chi3;
  }
  out->nwin = c.nwin;
  out->E0 = c.E0;
  out->t_peak = c.t0;
  std::vector<TableHost> none;
  Layout L;
  st = plan(cfg, c, none, &L);
  if (st != PIC_OK) return st;
  out->n_neutral = L.nneut;
  out->capacity = L.capacity;
  return PIC_OK;
}

pic_status pic_keldysh_rate(const pic_material* m, double lambda_m, int32_t terms, const double* A,
                            int64_t n, double* W_out) {
  if (!m || !A || !W_out || n < 0 || terms < 1 || !(lambda_m > 0)) return PIC_E_INVAL;
  MatC mc;
  mc.gap_eV = m->gap_eV;
  mc.n_index = m->n_index;
  mc.n0 = 0;
  mc.mred = 1.0 / (1.0 / m->me_star + 1.0 / m->mh_star);
  for (int64_t i = 0; i < n; ++i) W_out[i] = keldysh_W(mc, lambda_m, terms, A[i]);
  return PIC_OK;
}

static pic_status table_probe_host(const pic_config* cfg, int32_t mat, const float* A, int64_t n, float* out,
                                   bool bound) {
  if (!cfg || !A || !out || n < 0) return PIC_E_INVAL;
  Canon c;
  pic_status st = canonicalize(cfg, &c);
  if (st != PIC_OK) return st;
  TableHost T;
  st = build_table(c, mat, cfg->keldysh_terms, &T, cfg->keldysh_tol_bits > 0 ? cfg->keldysh_tol_bits : 60);
  if (st != PIC_OK) return st;
  const TabHdr* h = reinterpret_cast<const TabHdr*>(T.bytes.data());
  for (int64_t i = 0; i < n; ++i) out[i] = bound ? table_bound(h, A[i]) : table_lookup(h, A[i]);
  return PIC_OK;
}

pic_status pic_table_probe(const pic_config* cfg, int32_t mat, const float* A, int64_t n, float* P_out) {
  return table_probe_host(cfg, mat, A, n, P_out, false);
}

pic_status pic_table_bound_probe(const pic_config* cfg, int32_t mat, const float* A, int64_t n,
                                 float* B_out) {
  return table_probe_host(cfg, mat, A, n, B_out, true);
}

pic_status pic_footprint(const pic_config* cfg, size_t* bytes) {
  if (!cfg || !bytes) return PIC_E_INVAL;
  Canon c;
  pic_status st = canonicalize(cfg, &c);
  if (st != PIC_OK) return st;
  // tables: bounded estimate without building them (<= 1 MiB per material)
  std::vector<TableHost> est(c.nmat);
  for (auto& t : est) t.bytes.resize(1 << 20);
  Layout L;
  st = plan(cfg, c, est, &L);
  if (st != PIC_OK) return st;
  *bytes = L.total;
  return PIC_OK;
}

pic_status pic_init(const pic_config* cfg_in, pic_ctx** out) {
  if (!cfg_in || !out) return PIC_E_INVAL;
  *out = nullptr;
  (void)hipGetLastError();   // launch errors are checked below; drop stale ones
  pic_ctx* c = new (std::nothrow) pic_ctx();
  if (!c) return PIC_E_NOMEM;
  c->cfg = *cfg_in;
  pic_status st = canonicalize(cfg_in, &c->canon);
  if (st != PIC_OK) {
    delete c;
    return st;
  }
  c->mats.assign(cfg_in->mats, cfg_in->mats + cfg_in->nmat);
  c->layers.assign(cfg_in->layers, cfg_in->layers + cfg_in->nlayer);
  c->cfg.mats = c->mats.data();
  c->cfg.layers = c->layers.data();
  const Canon& K = c->canon;
  const int D = K.D;
  c->tabs.resize(K.nmat);
  for (int m = 0; m < K.nmat; ++m) {
    st = cached_table(K, m, cfg_in->keldysh_terms > 0 ? cfg_in->keldysh_terms : 500,
                      cfg_in->keldysh_tol_bits > 0 ? cfg_in->keldysh_tol_bits : 60, &c->tabs[m]);
    if (st != PIC_OK) {
      delete c;
      return st;
    }
  }
  st = plan(&c->cfg, K, c->tabs, &c->L);
  if (st != PIC_OK) {
    delete c;
    return st;
  }
  const Layout& L = c->L;
  c->stream = (hipStream_t)cfg_in->stream;
  void* mem = nullptr;
  if (cfg_in->alloc) {
    mem = cfg_in->alloc(L.total, cfg_in->alloc_user);
    c->owns_alloc_via_cb = 1;
  } else if (hipMalloc(&mem, L.total) != hipSuccess) {
    mem = nullptr;
  }
  if (!mem) {
    delete c;
    return PIC_E_NOMEM;
  }
  c->base = (unsigned char*)mem;
  auto fail = [&](pic_status s) {
    pic_destroy(c);
    return s;
  };
  {
    void* sp = nullptr;   // the allocation-free histogram's staging on this GPU
    if (scratch_ptr(&sp) != PIC_OK) return fail(PIC_E_DEVICE);
  }
  if (hipHostMalloc((void**)&c->h_step, sizeof(int)) != hipSuccess) return fail(PIC_E_NOMEM);
  if (hipMemsetAsync(c->base, 0, L.total, c->stream) != hipSuccess) return fail(PIC_E_DEVICE);

  // ---- host-built tables and parameter block
  std::vector<float> ie_half(L.Px, 1.0f), ie_node(L.Px, 1.0f);
  for (int64_t i = 0; i < K.n[0]; ++i)
    ie_half[i + G] = K.mat_cell[i] >= 0 ? K.mats[K.mat_cell[i]].ie : 1.0f;
  for (int64_t i = 0; i <= K.n[0]; ++i)
    ie_node[i + G] = K.mat_node[i] >= 0 ? K.mats[K.mat_node[i]].ie : 1.0f;
  const bool has_lor = L.lx0 < L.lx1;
  std::vector<float4> lor_half(has_lor ? L.Px : 0, make_float4(0.f, 0.f, 0.f, 0.f));
  std::vector<float4> lor_node(lor_half);
  auto lor_of = [&](int m) {
    return m >= 0 ? make_float4(K.mats[m].lor[0], K.mats[m].lor[1], K.mats[m].lor[2], K.mats[m].chi3)
                  : make_float4(0.f, 0.f, 0.f, 0.f);
  };
  if (has_lor) {
    for (int64_t i = 0; i < K.n[0]; ++i) lor_half[i + G] = lor_of(K.mat_cell[i]);
    for (int64_t i = 0; i <= K.n[0]; ++i) lor_node[i + G] = lor_of(K.mat_node[i]);
  }
  std::vector<float> src(4 * (size_t)L.nsrc, 0.0f);
  for (int m = 0; m < L.nsrc; ++m) {
    src[4 * m + 0] = (float)laser_field(K, m * K.dt);
    src[4 * m + 1] = (float)laser_field(K, m * K.dt - K.dx[0] / kC);
  }
  std::vector<float> prof((size_t)L.Py * L.Pz, 0.0f);
  for (int64_t k = 0; k < (D >= 3 ? K.n[2] + 1 : 1); ++k)
    for (int64_t j = 0; j < (D >= 2 ? K.n[1] + 1 : 1); ++j) {
      double y = 0.0, z = 0.0;
      if (D >= 2) y = ((double)j + (K.pol == 1 ? 0.5 : 0.0)) * K.dx[1] - 0.5 * K.n[1] * K.dx[1];
      if (D >= 3) z = ((double)k + (K.pol == 2 ? 0.5 : 0.0)) * K.dx[2] - 0.5 * K.n[2] * K.dx[2];
      prof[(D >= 2 ? j + G : 0) + L.Py * (D >= 3 ? k + G : 0)] = (float)transverse_profile(K, y, z);
    }
  c->mcell.clear();
  c->mcell.reserve(L.nmcell);
  for (int64_t k = 0; k < K.n[2]; ++k)
    for (int64_t j = 0; j < K.n[1]; ++j)
      for (int64_t i = 0; i < K.n[0]; ++i)
        if (K.mat_cell[i] >= 0) c->mcell.push_back(pack_cell(D, (int)i, (int)j, (int)k));

  Inst& I = c->h;
  std::memset(&I, 0, sizeof I);
  I.D = D;
  I.order = c->cfg.shape_order;
  I.nx = (int)K.n[0];
  I.ny = (int)K.n[1];
  I.nz = (int)K.n[2];
  I.Px = (int)L.Px;
  I.Py = (int)L.Py;
  I.Pz = (int)L.Pz;
  I.sy = (int)L.Px;
  I.sz = (int)(L.Px * L.Py);
  I.Gy = D >= 2 ? G : 0;
  I.Gz = D >= 3 ? G : 0;
  I.per_y = K.per[1];
  I.per_z = K.per[2];
  for (int d = 0; d < 3; ++d) {
    I.C[d] = K.C[d];
    I.halfC[d] = 0.5f * K.C[d];
    I.kmur[d] = K.kmur[d];
    I.dx[d] = K.dx[d];
  }
  I.vcell = K.vcell;
  I.ctdt_m = (float)(kC * K.dt);
  for (int par = 0; par < 2; ++par) {
    for (int q = 0; q < 6; ++q) I.F[par][q] = (float*)devp(c, L.o_F[par][q]);
    for (int q = 0; q < 3; ++q) I.Jb[par][q] = (float*)devp(c, L.o_J[par][q]);
  }
  I.ie_half = (const float*)devp(c, L.o_ie_half);
  I.ie_node = (const float*)devp(c, L.o_ie_node);
  c->col = ColBufs{};
  std::vector<int> mrank;
  if (K.collide || K.impact) {
    c->col.cnt = (int*)devp(c, L.o_ccnt);
    c->col.fill = (int*)devp(c, L.o_cfill);
    c->col.bsum = (int*)devp(c, L.o_cbsum);
    c->col.idx = (int*)devp(c, L.o_cidx);
    c->col.key = (uint64_t*)devp(c, L.o_ckey);
    c->col.active = (int*)devp(c, L.o_cact);
    const int nsb = col_scan_blocks((int)(K.n[0] * K.n[1] * K.n[2]) + 1);
    c->col.bact = c->col.active + (size_t)nsb * COL_SCAN_B;
    c->col.list = c->col.bact + nsb + 1;
    c->col.ncell = (int)(K.n[0] * K.n[1] * K.n[2]);
    c->col.dt = K.dt;
    c->col.nk = 2 * K.nmat;
    c->col.collide = K.collide;
    c->col.impact = K.impact;
    for (int m = 0; m < K.nmat; ++m) {
      c->col.imp_P[m] = K.mats[m].impact_P;
      c->col.imp_th[m] = K.mats[m].impact_th;
      c->col.gap[m] = K.mats[m].gap_eV * kQE;
    }
    // rank of each material x cell (the material cells run x fastest, then y, z)
    mrank.assign(K.n[0], -1);
    int r = 0;
    for (int64_t i = 0; i < K.n[0]; ++i)
      if (K.mat_cell[i] >= 0) mrank[i] = r++;
    c->col.nmx = r;
    c->col.mrank = (const int*)devp(c, L.o_mrank);
  }
  I.lx0 = L.lx0;
  I.lx1 = L.lx1;
  for (int par = 0; par < 2; ++par)
    for (int q = 0; q < 3; ++q) {
      I.Q[par][q] = has_lor ? (float*)devp(c, L.o_Q[par][q]) : nullptr;
      I.Kp[par][q] = has_lor ? (float*)devp(c, L.o_Kp[par][q]) : nullptr;
    }
  I.lor_half = has_lor ? (const float4*)devp(c, L.o_lor_half) : nullptr;
  I.lor_node = has_lor ? (const float4*)devp(c, L.o_lor_node) : nullptr;
  I.mat_cell = (const signed char*)devp(c, L.o_mat);
  I.pol = K.pol;
  I.nsrc = L.nsrc;
  I.src = (const float4*)devp(c, L.o_src);
  I.prof = (const float*)devp(c, L.o_prof);
  I.nwin = K.nwin;
  I.wx0 = L.wx0;
  I.wx1 = L.wx1;
  I.wnx = L.wx1 - L.wx0;
  I.wsz = L.wsz;
  I.ring = (float*)devp(c, L.o_ring);
  I.suffix = (float*)devp(c, L.o_suffix);
  I.prefix = (float*)devp(c, L.o_prefix);
  I.A = (float*)devp(c, L.o_A);
  I.pcell = (uint32_t*)devp(c, L.o_pcell);
  I.po0 = (uint32_t*)devp(c, L.o_po[0]);
  I.po1 = (uint32_t*)devp(c, L.o_po[1]);
  I.po2 = (uint32_t*)devp(c, L.o_po[2]);
  I.pu0 = (float*)devp(c, L.o_pu[0]);
  I.pu1 = (float*)devp(c, L.o_pu[1]);
  I.pu2 = (float*)devp(c, L.o_pu[2]);
  I.pkind = (uint8_t*)devp(c, L.o_pkind);
  I.pid = (uint32_t*)devp(c, L.o_pid);
  for (int d = 0; d < 3; ++d) I.ntile[d] = L.ntile[d];
  I.ntiles = (int)L.ntiles;
  I.tcnt = (int*)devp(c, L.o_tcnt);
  I.tstart = (int*)devp(c, L.o_tstart);
  I.tbirth = (int*)devp(c, L.o_tbirth);
  I.tslack = (int*)devp(c, L.o_tslack);
  I.tfill = (int*)devp(c, L.o_tfill);
  I.talive = (int*)devp(c, L.o_talive);
  I.tperm = (int*)devp(c, L.o_tperm);
  I.chunks = (int4*)devp(c, L.o_chunks);
  I.scell = (uint32_t*)devp(c, L.o_scell);
  I.so0 = (uint32_t*)devp(c, L.o_so[0]);
  I.so1 = (uint32_t*)devp(c, L.o_so[1]);
  I.so2 = (uint32_t*)devp(c, L.o_so[2]);
  I.su0 = (float*)devp(c, L.o_su[0]);
  I.su1 = (float*)devp(c, L.o_su[1]);
  I.su2 = (float*)devp(c, L.o_su[2]);
  I.skind = (uint8_t*)devp(c, L.o_skind);
  I.spid = (uint32_t*)devp(c, L.o_spid);
  c->d_ctr = (Ctr*)devp(c, L.o_ctr);
  I.pcount = &c->d_ctr->pcount;
  I.sctl = c->d_ctr->sctl;
  I.hot = c->d_ctr->hot;
  I.xext = c->d_ctr->xext;
  I.front = &c->d_ctr->front;
  I.tiles_done = c->d_ctr->tiles_done;
  I.step = &c->d_ctr->step;
  I.health = &c->d_ctr->health;
  I.nevents = c->d_ctr->nevents;
  I.pq = c->d_ctr->pq;
  I.eflux = c->d_ctr->eflux;
  for (int d = 0; d < 3; ++d) {
    // a plane normal to axis d: eps0 c dt times the transverse cell area
    // (absent axes count 1 m)
    double area = 1.0;
    for (int e = 0; e < D; ++e)
      if (e != d) area *= K.dx[e];
    I.kflux[d] = kEPS0 * kC * K.dt * area;
  }
  I.capacity = (int)L.capacity;
  for (int m = 0; m < K.nmat; ++m) {
    const MatC& mt = K.mats[m];
    const double kmass[2] = {mt.e_kg, mt.p_kg};
    for (int s = 0; s < 2; ++s) {
      const int kd = 2 * m + s;
      const double q = s == 0 ? -kQE : kQE;
      const double qhat = q * mt.n0 / (K.ppc > 0 ? K.ppc : 1) / kEPS0;
      I.kh[kd] = (float)(q * K.dt / (2.0 * kmass[s] * kC));
      for (int d = 0; d < 3; ++d) I.kq[kd][d] = (float)(d < D ? qhat * K.dx[d] : qhat * kC * K.dt);
      I.kqhat[kd] = qhat;
      I.kw[kd] = mt.n0 * K.vcell / (K.ppc > 0 ? K.ppc : 1);
      I.kmass[kd] = kmass[s];
    }
    I.ksig[m] = (float)(std::sqrt(kKB * c->cfg.T_K / mt.mol_kg) / kC);
    I.tab[m] = (const TabHdr*)devp(c, L.o_tab[m]);
    I.acut[m] = c->tabs[m].acut;
  }
  I.nmat = K.nmat;
  I.acut_min = 3.0e38f;
  for (int m = 0; m < K.nmat; ++m) I.acut_min = std::min(I.acut_min, I.acut[m]);
  // fixed-point scale of the LDS deposit: 2^JFIX_BITS per 2^ceil(log2 max |kq|)
  float qmax = 0.0f;
  for (int kd = 0; kd < 2 * K.nmat; ++kd)
    for (int d = 0; d < 3; ++d) qmax = std::max(qmax, std::fabs(I.kq[kd][d]));
  const int qexp = qmax > 0.0f ? (int)std::ceil(std::log2((double)qmax)) : 0;
  I.jscale = std::ldexp(1.0f, JFIX_BITS - qexp);
  I.jscale_inv = std::ldexp(1.0f, qexp - JFIX_BITS);
  I.nneut = L.nneut;
  I.ppc = K.ppc;
  I.ppc_magic = K.ppc > 1 ? UINT64_MAX / (uint64_t)K.ppc + 1 : 0;
  I.no0 = (float*)devp(c, L.o_no[0]);
  I.no1 = (float*)devp(c, L.o_no[1]);
  I.no2 = (float*)devp(c, L.o_no[2]);
  I.alive = (uint32_t*)devp(c, L.o_alive);
  I.death = (int*)devp(c, L.o_death);
  I.mcell = (const uint32_t*)devp(c, L.o_mcell);
  I.seed = c->cfg.seed;
  c->d_inst = (Inst*)devp(c, L.o_inst);
  c->d_off = (int*)devp(c, L.o_off);
  c->d_off_fields = c->d_off + 2;
  c->d_grid64 = (double*)devp(c, L.o_grid64);

  // block counts per phase
  auto nblk = [](int64_t n) { return (int)std::max<int64_t>(0, (n + TPB - 1) / TPB); };
  c->nb_push = push_grid(D);
  if (c->nb_push <= 0) return fail(PIC_E_DEVICE);
  // field tile shape: default per dimension (the shapes the in-run timing
  // picks on MI355X for the benchmark grids: 60x8 in 2D, 12x8x4 in 3D),
  // overridable (tuning sweeps) by PIC_FIELD_TILE=<variant>
  c->tile = D == 2 ? 5 : (D == 3 ? 6 : 0);
  c->nvar = field_tile_variants(D, c->canon.per[1] && (D < 3 || c->canon.per[2]));
  if (const char* tv = std::getenv("PIC_FIELD_TILE")) c->tile = std::max(0, std::min(atoi(tv), c->nvar - 1));
  c->nb_cell = field_tiles(D, c->tile, (int)L.Px, (int)L.Py, (int)L.Pz);
  c->nb_win = 1;   // one block per instance (tile-sort scan)
  {
    const int64_t span = (int64_t)TPB * ion_nit(K.ppc);
    c->nb_neut = (int)std::max<int64_t>(1, (L.nneut + span - 1) / span);
  }

  c->nb_sort = sort_blocks(L.capacity);
  int offs[32] = {0, c->nb_push, 0, c->nb_cell, 0, c->nb_win, 0, c->nb_neut};
  offs[2 * PH_SORT + 1] = c->nb_sort;
  for (int v = 0; v < c->nvar; ++v)
    offs[9 + 2 * v] = field_tiles(D, v, (int)L.Px, (int)L.Py, (int)L.Pz);

  hipStream_t s = c->stream;
  bool ok = true;
  ok &= hipMemcpyAsync(devp(c, L.o_ie_half), ie_half.data(), sizeof(float) * L.Px, hipMemcpyHostToDevice, s) == hipSuccess;
  ok &= hipMemcpyAsync(devp(c, L.o_ie_node), ie_node.data(), sizeof(float) * L.Px, hipMemcpyHostToDevice, s) == hipSuccess;
  if (has_lor) {
    ok &= hipMemcpyAsync(devp(c, L.o_lor_half), lor_half.data(), sizeof(float4) * L.Px, hipMemcpyHostToDevice, s) ==
          hipSuccess;
    ok &= hipMemcpyAsync(devp(c, L.o_lor_node), lor_node.data(), sizeof(float4) * L.Px, hipMemcpyHostToDevice, s) ==
          hipSuccess;
  }
  ok &= hipMemcpyAsync(devp(c, L.o_mat), K.mat_cell.data(), K.n[0], hipMemcpyHostToDevice, s) == hipSuccess;
  if (!mrank.empty())
    ok &= hipMemcpyAsync(devp(c, L.o_mrank), mrank.data(), sizeof(int) * mrank.size(), hipMemcpyHostToDevice, s) ==
          hipSuccess;
  ok &= hipMemcpyAsync(devp(c, L.o_src), src.data(), sizeof(float) * src.size(), hipMemcpyHostToDevice, s) == hipSuccess;
  ok &= hipMemcpyAsync(devp(c, L.o_prof), prof.data(), sizeof(float) * prof.size(), hipMemcpyHostToDevice, s) == hipSuccess;
  if (!c->mcell.empty())
    ok &= hipMemcpyAsync(devp(c, L.o_mcell), c->mcell.data(), sizeof(uint32_t) * c->mcell.size(),
                         hipMemcpyHostToDevice, s) == hipSuccess;
  for (int m = 0; m < K.nmat; ++m)
    ok &= hipMemcpyAsync(devp(c, L.o_tab[m]), c->tabs[m].bytes.data(), c->tabs[m].bytes.size(),
                         hipMemcpyHostToDevice, s) == hipSuccess;
  ok &= hipMemcpyAsync(c->d_inst, &I, sizeof I, hipMemcpyHostToDevice, s) == hipSuccess;
  ok &= hipMemcpyAsync(c->d_off, offs, sizeof offs, hipMemcpyHostToDevice, s) == hipSuccess;
  float sig[2 * MAXMAT] = {0};
  if (c->cfg.preionize_eV > 0) {
    for (int m = 0; m < K.nmat; ++m) {
      sig[m] = (float)(std::sqrt(c->cfg.preionize_eV * kQE / K.mats[m].e_kg) / kC);
      sig[MAXMAT + m] = (float)(std::sqrt(c->cfg.preionize_eV * kQE / K.mats[m].p_kg) / kC);
    }
    ok &= hipMemcpyAsync(devp(c, L.o_sig), sig, sizeof sig, hipMemcpyHostToDevice, s) == hipSuccess;
  }
  if (!ok) return fail(PIC_E_DEVICE);
  // alive neutrals per particle tile (the bound the birth room is sized by)
  // and a sort at the first check, which lays the tiles and their birth room out
  {
    std::vector<int> talive(L.ntiles, 0);
    if (c->cfg.preionize_eV <= 0) {
      for (uint32_t pc : c->mcell) {
        int ci, cj, ck;
        unpack_cell(D, pc, ci, cj, ck);
        int64_t t = ci / ptile_ext(D, 0);
        if (D >= 2) t += (int64_t)L.ntile[0] * (cj / ptile_ext(D, 1));
        if (D >= 3) t += (int64_t)L.ntile[0] * L.ntile[1] * (ck / ptile_ext(D, 2));
        talive[t] += K.ppc;
      }
    }
    ok &= hipMemcpyAsync(devp(c, L.o_talive), talive.data(), sizeof(int) * L.ntiles, hipMemcpyHostToDevice,
                         s) == hipSuccess;
    if (c->cfg.preionize_eV <= 0 && L.nneut > 0) {
      static const int force = 1;
      ok &= hipMemcpyAsync(&c->d_ctr->sctl[SC_FORCE], &force, sizeof force, hipMemcpyHostToDevice, s) ==
            hipSuccess;
    }
  }
  // charged region: the amplitude window (births and preionized carriers are
  // all inside it)
  set_region(c, 1 << 30, -(1 << 30));
  ok &= hipMemcpyAsync(c->d_ctr->xext, c->h_xext, sizeof c->h_xext, hipMemcpyHostToDevice, s) == hipSuccess;
  if (!ok) return fail(PIC_E_DEVICE);
  launch_init_neutrals_d(c->d_inst, L.nneut, D, s);
  if (c->cfg.preionize_eV > 0 && L.nneut > 0) {
    const float* sg = (const float*)devp(c, L.o_sig);
    launch_preionize_d(c->d_inst, L.nneut, D, sg, sg + MAXMAT, s);
    const int cnt = (int)(2 * L.nneut);
    if (hipMemcpyAsync(&c->d_ctr->pcount, &cnt, sizeof cnt, hipMemcpyHostToDevice, s) != hipSuccess)
      return fail(PIC_E_DEVICE);
  }
  if (hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess) return fail(PIC_E_DEVICE);
  *out = c;
  return PIC_OK;
}

void pic_destroy(pic_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream); else (void)hipDeviceSynchronize();
  for (int ph = 0; ph < 8; ++ph)
    for (int k = 0; k < pic_ctx::kRing; ++k)
      for (int e = 0; e < 2; ++e)
        if (c->ev[ph][k][e]) (void)hipEventDestroy(c->ev[ph][k][e]);
  for (auto& vv : c->tune_ev)
    for (auto& rr : vv)
      for (auto& e : rr)
        if (e) (void)hipEventDestroy(e);
  if (c->h_step) (void)hipHostFree(c->h_step);
  dev_free(c, c->d_imax);
  dev_free(c, c->d_spec);
  dev_free(c, c->d_tracks);
  if (c->base) {
    if (c->owns_alloc_via_cb && c->cfg.free) c->cfg.free(c->base, c->cfg.alloc_user);
    else if (!c->owns_alloc_via_cb) (void)hipFree(c->base);
  }
  delete c;
}

// ------------------------------------------------------------ checkpoints
namespace {
struct SnapHdr {
  uint64_t magic;      // "PICSNAP1"
  uint32_t version, hdr_bytes;
  uint64_t total;      // bytes of the device state block that follow
  uint64_t key;        // hash of the layout and the canonical problem
  int64_t step;
  int32_t tile, nb_cell, far_skip, resort;
  int32_t xext[6];
};
constexpr uint64_t kSnapMagic = 0x31504e5350434950ull;   // "PICSNAP1"

// FNV-1a over the quantities that fix the state block's layout and meaning
uint64_t snap_key(const pic_ctx* c) {
  const Layout& L = c->L;
  const Canon& K = c->canon;
  const double v[] = {(double)L.total, (double)L.ncell, (double)L.nneut, (double)L.capacity,
                      (double)L.Px, (double)L.Py, (double)L.Pz, (double)L.nmcell, (double)L.o_inst,
                      K.dt, K.dx[0], K.dx[1], K.dx[2], (double)K.ppc, (double)K.nmat,
                      (double)c->cfg.seed, (double)c->cfg.shape_order};
  uint64_t h = 1469598103934665603ull;
  const unsigned char* p = reinterpret_cast<const unsigned char*>(v);
  for (size_t i = 0; i < sizeof v; ++i) h = (h ^ p[i]) * 1099511628211ull;
  return h;
}
}  // namespace

pic_status pic_snapshot(pic_ctx* c, void* host_out, size_t out_bytes, size_t* written) {
  if (!c) return PIC_E_INVAL;
  const Layout& L = c->L;
  const size_t need = sizeof(SnapHdr) + (size_t)L.total;
  if (written) *written = need;
  if (!host_out) return PIC_OK;
  if (out_bytes < need) return PIC_E_INVAL;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return PIC_E_DEVICE;
  SnapHdr h{};
  h.magic = kSnapMagic;
  h.version = 1;
  h.hdr_bytes = sizeof(SnapHdr);
  h.total = (uint64_t)L.total;
  h.key = snap_key(c);
  h.step = c->step;
  h.tile = c->tile;
  h.nb_cell = c->nb_cell;
  h.far_skip = c->far_skip;
  h.resort = c->resort;
  for (int q = 0; q < 6; ++q) h.xext[q] = c->h_xext[q];
  std::memcpy(host_out, &h, sizeof h);
  HIP_OK(hipMemcpy((unsigned char*)host_out + sizeof h, c->base, (size_t)L.total, hipMemcpyDeviceToHost));
  return PIC_OK;
}

pic_status pic_restore(pic_ctx* c, const void* host_in, size_t in_bytes) {
  if (!c || !host_in || in_bytes < sizeof(SnapHdr)) return PIC_E_INVAL;
  SnapHdr h;
  std::memcpy(&h, host_in, sizeof h);
  if (h.magic != kSnapMagic || h.version != 1 || h.hdr_bytes != sizeof(SnapHdr)) return PIC_E_VERSION;
  const Layout& L = c->L;
  if (h.total != (uint64_t)L.total || h.key != snap_key(c) || in_bytes < sizeof h + (size_t)L.total ||
      h.tile < 0 || h.tile >= c->nvar)
    return PIC_E_INVAL;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return PIC_E_DEVICE;
  harvest_all(c);
  // every byte of the state block except this context's own parameter block,
  // which holds its device addresses
  const unsigned char* src = (const unsigned char*)host_in + sizeof h;
  const size_t i0 = L.o_inst, i1 = L.o_inst + sizeof(Inst);
  HIP_OK(hipMemcpy(c->base, src, i0, hipMemcpyHostToDevice));
  if ((size_t)L.total > i1) HIP_OK(hipMemcpy(c->base + i1, src + i1, (size_t)L.total - i1, hipMemcpyHostToDevice));
  c->step = h.step;
  c->tile = h.tile;
  c->nb_cell = h.nb_cell;
  c->d_off_fields = c->d_off + 8 + 2 * c->tile;
  c->tune_left = 0;
  c->far_skip = h.far_skip;
  c->resort = h.resort;
  for (int q = 0; q < 6; ++q) c->h_xext[q] = h.xext[q];
  c->latched = PIC_OK;
  check_health(c);
  return PIC_OK;
}

pic_status pic_set_imax(pic_ctx* c, int32_t every) {
  if (!c || every < 0) return PIC_E_INVAL;
  if (c->latched != PIC_OK) return PIC_E_STATE;
  if (every > 0) {
    const size_t bytes = sizeof(float) * c->L.ncell;
    if (!c->d_imax) {
      c->d_imax = (float*)dev_alloc(c, bytes);
      if (!c->d_imax) return PIC_E_NOMEM;
    }
    HIP_OK(hipMemsetAsync(c->d_imax, 0, bytes, c->stream));
  }
  c->imax_every = every;
  return PIC_OK;
}

pic_status pic_spectrum_counts(pic_ctx* c, const pic_spectrum* sp, uint64_t* out, size_t out_count) {
  pic_status st = spectrum_check(c, sp, out, out_count);
  if (st != PIC_OK) return st;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return PIC_E_DEVICE;
  if (!c->d_spec) {
    c->d_spec = dev_alloc(c, kSpecBytes);
    if (!c->d_spec) return PIC_E_NOMEM;
  }
  return spectrum_into(c, sp, out, out_count, c->d_spec);
}

pic_status pic_spectrum_counts_noalloc(pic_ctx* c, const pic_spectrum* sp, uint64_t* out, size_t out_count) {
  pic_status st = spectrum_check(c, sp, out, out_count);
  if (st != PIC_OK) return st;
  void* buf = nullptr;
  st = scratch_ptr(&buf);
  if (st != PIC_OK) return st;
  return spectrum_into(c, sp, out, out_count, buf);
}

pic_status pic_set_tracks(pic_ctx* c, uint32_t threshold, int32_t every, int64_t max_records) {
  if (!c || every < 0 || max_records < 0) return PIC_E_INVAL;
  if (c->latched != PIC_OK) return PIC_E_STATE;
  if (every > 0) {
    // ids are stored in 32 bits: neutral ids and placed particles' ids must fit
    if ((double)placed_id_base(c) + (double)c->L.capacity > 4294967295.0) return PIC_E_INVAL;
    if (max_records > ((int64_t)1 << 40) / (int64_t)sizeof(TrackRec)) return PIC_E_INVAL;
    const size_t bytes = 256 + sizeof(TrackRec) * (size_t)max_records;
    if (c->d_tracks && c->track_max != max_records) {
      if (hipStreamSynchronize(c->stream) != hipSuccess) return PIC_E_DEVICE;
      dev_free(c, c->d_tracks);
      c->d_tracks = nullptr;
    }
    if (!c->d_tracks) {
      c->d_tracks = dev_alloc(c, bytes);
      if (!c->d_tracks) return PIC_E_NOMEM;
    }
    c->track_max = max_records;
    HIP_OK(hipMemsetAsync(c->d_tracks, 0, 256, c->stream));
  }
  c->track_every = every;
  c->track_thr = threshold;
  return PIC_OK;
}

pic_status pic_set_timing(pic_ctx* c, int32_t on) {
  if (!c) return PIC_E_INVAL;
  harvest_all(c);
  c->timing = on;
  for (int ph = 0; ph < 8; ++ph) c->timers[ph] = c->tcount[ph] = 0.0;
  return PIC_OK;
}

pic_status pic_set_far_tiles(pic_ctx* c, int32_t on) {
  if (!c) return PIC_E_INVAL;
  c->far_skip = on ? 1 : 0;
  return PIC_OK;
}

pic_status pic_set_resort(pic_ctx* c, int32_t period) {
  if (!c || period < 0) return PIC_E_INVAL;
  c->resort = period;
  return PIC_OK;
}

pic_status pic_step(pic_ctx* c, int64_t nsteps) {
  if (!c || nsteps < 0) return PIC_E_INVAL;
  if (c->latched != PIC_OK) return PIC_E_STATE;
  (void)hipGetLastError();
  for (int64_t s = 0; s < nsteps; ++s) enqueue_step(c);   // advances c->step
  // keep the device step counter (read by batches and diagnostics) in step
  *c->h_step = (int)c->step;
  (void)hipMemcpyAsync(&c->d_ctr->step, c->h_step, sizeof(int), hipMemcpyHostToDevice, c->stream);
  if (hipGetLastError() != hipSuccess) return PIC_E_DEVICE;
  return PIC_OK;
}

// Field-kernel tile autotuner: before the first step the fields, currents and
// amplitude window are all zero, so every variant can be timed on the real
// launch shape; the state is cleared again afterwards (exactly the initial state).
// Lorentz media back at rest (Q = K = 0 in both sets); stream null: synchronous
hipError_t clear_polarisation(pic_ctx* c, hipStream_t s) {
  const Layout& L = c->L;
  if (L.lx0 >= L.lx1) return hipSuccess;
  for (int par = 0; par < 2; ++par)
    for (int q = 0; q < 3; ++q)
      for (void* p : {devp(c, L.o_Q[par][q]), devp(c, L.o_Kp[par][q])}) {
        const hipError_t e = s ? hipMemsetAsync(p, 0, sizeof(float) * L.ncell, s)
                               : hipMemset(p, 0, sizeof(float) * L.ncell);
        if (e != hipSuccess) return e;
      }
  return hipSuccess;
}

pic_status pic_autotune(pic_ctx* c, int32_t reps) {
  if (!c || reps < 1) return PIC_E_INVAL;
  if (c->step != 0 || c->cfg.preionize_eV > 0) return PIC_E_STATE;
  const Layout& L = c->L;
  const int D = c->canon.D;
  hipStream_t s = c->stream;
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  double best = 1e30;
  int best_v = c->tile;
  int offs[2];
  // three interleaved rounds over the tile shapes, best round of each kept
  // (the differences are a few percent, close to the launch-to-launch noise)
  for (int v = 0; v < c->nvar; ++v) c->tune_ms[v] = 1e30;
  for (int round = 0; round < 3; ++round) {
    for (int v = 0; v < c->nvar; ++v) {
      const int nb = field_tiles(D, v, (int)L.Px, (int)L.Py, (int)L.Pz);
      offs[0] = 0;
      offs[1] = nb;
      HIP_OK(hipMemcpy(c->d_off + 2, offs, sizeof offs, hipMemcpyHostToDevice));
      Group gr{c->d_inst, c->d_off + 2, 1, nb, 0};
      gr.front = &c->d_ctr->front;
      gr.xext = c->d_ctr->xext;
      gr.host = &c->h;
      gr.lor = disp_mode(c->L);
      launch_fields(gr, D, v, s);   // warm
      HIP_OK(hipEventRecord(e0, s));
      for (int r = 0; r < reps; ++r) launch_fields(gr, D, v, s);
      HIP_OK(hipEventRecord(e1, s));
      HIP_OK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_OK(hipEventElapsedTime(&ms, e0, e1));
      c->tune_ms[v] = std::min(c->tune_ms[v], (double)ms / reps);
    }
  }
  for (int v = 0; v < c->nvar; ++v)
    if (c->tune_ms[v] < best) {
      best = c->tune_ms[v];
      best_v = v;
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->tile = best_v;
  c->nb_cell = field_tiles(D, best_v, (int)L.Px, (int)L.Py, (int)L.Pz);
  offs[0] = 0;
  offs[1] = c->nb_cell;
  HIP_OK(hipMemcpy(c->d_off + 2, offs, sizeof offs, hipMemcpyHostToDevice));
  // back to the initial state: fields, currents, window and amplitude zero
  for (int par = 0; par < 2; ++par) {
    for (int q = 0; q < 6; ++q) HIP_OK(hipMemsetAsync(devp(c, L.o_F[par][q]), 0, sizeof(float) * L.ncell, s));
    for (int q = 0; q < 3; ++q) HIP_OK(hipMemsetAsync(devp(c, L.o_J[par][q]), 0, sizeof(float) * L.ncell, s));
  }
  HIP_OK(clear_polarisation(c, s));
  HIP_OK(hipMemsetAsync(devp(c, L.o_ring), 0, sizeof(float) * L.wsz * c->canon.nwin, s));
  HIP_OK(hipMemsetAsync(devp(c, L.o_suffix), 0, sizeof(float) * L.wsz * c->canon.nwin, s));
  HIP_OK(hipMemsetAsync(devp(c, L.o_prefix), 0, sizeof(float) * L.wsz, s));
  HIP_OK(hipMemsetAsync(devp(c, L.o_A), 0, sizeof(float) * L.ncell, s));
  HIP_OK(hipMemsetAsync(&c->d_ctr->health, 0, sizeof(unsigned), s));
  HIP_OK(hipMemsetAsync(c->d_ctr->hot, 0, sizeof(c->d_ctr->hot), s));
  HIP_OK(hipMemsetAsync(&c->d_ctr->front, 0, sizeof(int), s));
  HIP_OK(hipStreamSynchronize(s));
  return PIC_OK;
}

pic_status pic_autotune_steps(pic_ctx* c, int32_t reps) {
  if (!c || reps < 1 || reps > 16) return PIC_E_INVAL;
  if (c->tune_left > 0) return PIC_E_STATE;
  for (int v = 0; v < c->nvar; ++v)
    for (int r = 0; r < reps; ++r)
      for (int e = 0; e < 2; ++e)
        if (!c->tune_ev[v][r][e]) HIP_OK(timing_event(&c->tune_ev[v][r][e]));
  c->tune_reps = reps;
  c->tune_left = c->nvar * reps;
  return PIC_OK;
}

pic_status pic_set_state(pic_ctx* c, const pic_state* S) {
  if (!c || !S) return PIC_E_INVAL;
  if (S->n_particles < 0 || S->n_particles > c->L.capacity || (S->n_particles > 0 && !S->particles))
    return PIC_E_INVAL;
  const Canon& K = c->canon;
  const Layout& L = c->L;
  const int D = K.D;
  hipStream_t s = c->stream;
  if (hipStreamSynchronize(s) != hipSuccess) return PIC_E_DEVICE;
  std::vector<float> buf(L.ncell);
  const int spar = (int)(S->step & 1);
  for (int w = 0; w < 2; ++w)
    for (int q = 0; q < 3; ++q) {
      const float* src = w == 0 ? S->E[q] : S->b[q];
      if (!src) continue;
      std::fill(buf.begin(), buf.end(), 0.0f);
      const bool* half = w == 0 ? kHalfE[q] : kHalfB[q];
      for_domain(K, half, [&](int64_t n, int64_t i, int64_t j, int64_t k) { buf[pidx(L, D, i, j, k)] = src[n]; });
      HIP_OK(hipMemcpy(devp(c, L.o_F[spar][3 * w + q]), buf.data(), sizeof(float) * L.ncell,
                       hipMemcpyHostToDevice));
    }
  const int64_t n = S->n_particles;
  if (n > 0 || true) {
    std::vector<uint32_t> pc(n);
    std::vector<uint32_t> po[3];
    std::vector<float> pu[3];
    for (int q = 0; q < 3; ++q) {
      po[q].resize(n);
      pu[q].resize(n);
    }
    std::vector<uint8_t> pk(n);
    std::vector<uint32_t> pid(n);
    const int64_t id0 = placed_id_base(c);
    for (int64_t p = 0; p < n; ++p) {
      pid[p] = (uint32_t)(id0 + p);
      const pic_particle& r = S->particles[p];
      for (int d = 0; d < D; ++d)
        if (r.cell[d] < 0 || r.cell[d] >= K.n[d] || !(r.off[d] >= 0.0f && r.off[d] < 1.0f)) return PIC_E_INVAL;
      if (r.kind < 0 || r.kind >= 2 * K.nmat) return PIC_E_INVAL;
      pc[p] = pack_cell(D, r.cell[0], D >= 2 ? r.cell[1] : 0, D >= 3 ? r.cell[2] : 0);
      for (int q = 0; q < 3; ++q) {
        po[q][p] = q < D ? off_fix(r.off[q]) : 0u;
        pu[q][p] = r.u[q];
      }
      pk[p] = (uint8_t)r.kind;
    }
    if (n > 0) {
      HIP_OK(hipMemcpy(devp(c, L.o_pcell), pc.data(), 4 * n, hipMemcpyHostToDevice));
      for (int q = 0; q < 3; ++q) {
        if (q < D) HIP_OK(hipMemcpy(devp(c, L.o_po[q]), po[q].data(), 4 * n, hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(devp(c, L.o_pu[q]), pu[q].data(), 4 * n, hipMemcpyHostToDevice));
      }
      HIP_OK(hipMemcpy(devp(c, L.o_pkind), pk.data(), n, hipMemcpyHostToDevice));
      HIP_OK(hipMemcpy(devp(c, L.o_pid), pid.data(), 4 * n, hipMemcpyHostToDevice));
    }
    const int cnt = (int)n;
    HIP_OK(hipMemcpy(&c->d_ctr->pcount, &cnt, sizeof cnt, hipMemcpyHostToDevice));
    int lo = 1 << 30, hi = -(1 << 30);
    for (int64_t p = 0; p < n; ++p) {
      lo = std::min(lo, S->particles[p].cell[0]);
      hi = std::max(hi, S->particles[p].cell[0]);
    }
    set_region(c, lo, hi);
    HIP_OK(hipMemcpy(c->d_ctr->xext, c->h_xext, sizeof c->h_xext, hipMemcpyHostToDevice));
    // the new fields may be nonzero anywhere: no tile is beyond the field front
    const int fr = (int)L.Px;
    HIP_OK(hipMemcpy(&c->d_ctr->front, &fr, sizeof fr, hipMemcpyHostToDevice));
    // the new particles are all unsorted
    HIP_OK(hipMemset(c->d_ctr->sctl, 0, sizeof(c->d_ctr->sctl)));
    // no birth room until the next sort lays the tiles out again
    HIP_OK(hipMemset(devp(c, L.o_tslack), 0, sizeof(int) * L.ntiles));
  }
  const int st = (int)S->step;
  HIP_OK(hipMemcpy(&c->d_ctr->step, &st, sizeof st, hipMemcpyHostToDevice));
  c->step = S->step;
  if (S->reset_window) {
    HIP_OK(hipMemset(devp(c, L.o_ring), 0, sizeof(float) * L.wsz * K.nwin));
    HIP_OK(hipMemset(devp(c, L.o_suffix), 0, sizeof(float) * L.wsz * K.nwin));
    HIP_OK(hipMemset(devp(c, L.o_prefix), 0, sizeof(float) * L.wsz));
    HIP_OK(hipMemset(devp(c, L.o_A), 0, sizeof(float) * L.ncell));
  }
  for (int par = 0; par < 2; ++par)
    for (int q = 0; q < 3; ++q) HIP_OK(hipMemset(devp(c, L.o_J[par][q]), 0, sizeof(float) * L.ncell));
  HIP_OK(clear_polarisation(c, nullptr));
  HIP_OK(hipDeviceSynchronize());
  return PIC_OK;
}

pic_status pic_diag(pic_ctx* c, int kind, void* host_out, size_t out_bytes, size_t* written) {
  if (!c) return PIC_E_INVAL;
  const Canon& K = c->canon;
  const Layout& L = c->L;
  const int D = K.D;
  hipStream_t s = c->stream;
  if (hipStreamSynchronize(s) != hipSuccess) return PIC_E_DEVICE;
  check_health(c);
  size_t need = 0;
  switch (kind) {
    case PIC_DIAG_SCALARS: need = sizeof(double) * PIC_SC_COUNT; break;
    case PIC_DIAG_FIELDS: {
      for (int q = 0; q < 3; ++q) need += sizeof(double) * (dom_count(K, kHalfE[q]) + dom_count(K, kHalfB[q]));
      break;
    }
    case PIC_DIAG_POL: {
      for (int q = 0; q < 3; ++q) need += 2 * sizeof(double) * dom_count(K, kHalfE[q]);
      break;
    }
    case PIC_DIAG_NE_GRID:
    case PIC_DIAG_UE_GRID: need = sizeof(double) * dom_count(K, kNode); break;
    case PIC_DIAG_AMP:
    case PIC_DIAG_IMAX: need = sizeof(float) * dom_count(K, kNode); break;
    case PIC_DIAG_PARAMS: need = sizeof(pic_params); break;
    case PIC_DIAG_TIMERS: need = sizeof(double) * 32; break;
    case PIC_DIAG_SORT: need = sizeof(double) * 4; break;
    case PIC_DIAG_REGION: need = sizeof(double) * 6; break;
    case PIC_DIAG_HEALTH: need = sizeof(double) * 4; break;
    case PIC_DIAG_EVENTS:
    case PIC_DIAG_TRACKS:
    case PIC_DIAG_PARTICLES: break;   // computed below
    default: return PIC_E_INVAL;
  }
  if (kind == PIC_DIAG_EVENTS) {
    std::vector<int> death(L.nneut);
    if (L.nneut) HIP_OK(hipMemcpy(death.data(), devp(c, L.o_death), 4 * L.nneut, hipMemcpyDeviceToHost));
    std::vector<int64_t> pairs;
    for (int64_t jn = 0; jn < L.nneut; ++jn) {
      if (death[jn] < 0) continue;
      const int64_t m = jn / K.ppc, kk = jn - m * K.ppc;
      int ci, cj, ck;
      unpack_cell(D, c->mcell[m], ci, cj, ck);
      const int64_t lin = ci + K.n[0] * (cj + K.n[1] * (int64_t)ck);
      pairs.push_back(lin * K.ppc + kk);
      pairs.push_back(death[jn]);
    }
    need = sizeof(int64_t) * pairs.size();
    if (written) *written = need;
    if (!host_out) return PIC_OK;
    if (out_bytes < need) return PIC_E_INVAL;
    if (need) std::memcpy(host_out, pairs.data(), need);
    return PIC_OK;
  }
  if (kind == PIC_DIAG_TRACKS) {
    unsigned long long nrec = 0;
    if (c->d_tracks) HIP_OK(hipMemcpy(&nrec, c->d_tracks, sizeof nrec, hipMemcpyDeviceToHost));
    const int64_t keep = std::min<int64_t>((int64_t)nrec, c->track_max);
    need = sizeof(TrackRec) * (size_t)keep;
    if (written) *written = need;
    if (!host_out) return PIC_OK;
    if (out_bytes < need) return PIC_E_INVAL;
    if (keep > 0) {
      TrackRec* o = (TrackRec*)host_out;
      HIP_OK(hipMemcpy(o, (unsigned char*)c->d_tracks + 256, need, hipMemcpyDeviceToHost));
      std::sort(o, o + keep, [](const TrackRec& a, const TrackRec& b) {
        if (a.id != b.id) return a.id < b.id;
        if (a.kind != b.kind) return a.kind < b.kind;
        return a.step < b.step;
      });
    }
    return PIC_OK;
  }
  if (kind == PIC_DIAG_PARTICLES) {
    int cnt = 0;
    HIP_OK(hipMemcpy(&cnt, &c->d_ctr->pcount, sizeof cnt, hipMemcpyDeviceToHost));
    cnt = std::min<int64_t>(cnt, L.capacity);
    std::vector<uint32_t> pc(cnt);
    std::vector<uint32_t> po[3];
    std::vector<float> pu[3];
    std::vector<uint8_t> pk(cnt);
    if (cnt) {
      HIP_OK(hipMemcpy(pc.data(), devp(c, L.o_pcell), 4 * cnt, hipMemcpyDeviceToHost));
      HIP_OK(hipMemcpy(pk.data(), devp(c, L.o_pkind), cnt, hipMemcpyDeviceToHost));
    }
    for (int q = 0; q < 3; ++q) {
      po[q].assign(cnt, 0u);
      pu[q].resize(cnt);
      if (cnt && q < D) HIP_OK(hipMemcpy(po[q].data(), devp(c, L.o_po[q]), 4 * cnt, hipMemcpyDeviceToHost));
      if (cnt) HIP_OK(hipMemcpy(pu[q].data(), devp(c, L.o_pu[q]), 4 * cnt, hipMemcpyDeviceToHost));
    }
    std::vector<pic_particle> recs;
    for (int p = 0; p < cnt; ++p) {
      if (pk[p] == DEAD) continue;
      pic_particle r{};
      int ci, cj, ck;
      unpack_cell(D, pc[p], ci, cj, ck);
      r.cell[0] = ci;
      r.cell[1] = cj;
      r.cell[2] = ck;
      r.kind = pk[p];
      for (int q = 0; q < 3; ++q) {
        r.off[q] = q < D ? off_f32(po[q][p]) : 0.0f;
        r.u[q] = pu[q][p];
      }
      recs.push_back(r);
    }
    need = sizeof(pic_particle) * recs.size();
    if (written) *written = need;
    if (!host_out) return PIC_OK;
    if (out_bytes < need) return PIC_E_INVAL;
    if (need) std::memcpy(host_out, recs.data(), need);
    return PIC_OK;
  }
  if (written) *written = need;
  if (!host_out) return PIC_OK;
  if (out_bytes < need) return PIC_E_INVAL;

  if (kind == PIC_DIAG_FIELDS) {
    double* o = (double*)host_out;
    std::vector<float> buf(L.ncell);
    int dstep = 0;
    HIP_OK(hipMemcpy(&dstep, &c->d_ctr->step, sizeof dstep, hipMemcpyDeviceToHost));
    for (int w = 0; w < 2; ++w)
      for (int q = 0; q < 3; ++q) {
        HIP_OK(hipMemcpy(buf.data(), devp(c, L.o_F[dstep & 1][3 * w + q]), sizeof(float) * L.ncell,
                         hipMemcpyDeviceToHost));
        const bool* half = w == 0 ? kHalfE[q] : kHalfB[q];
        for_domain(K, half, [&](int64_t n, int64_t i, int64_t j, int64_t k) { o[n] = buf[pidx(L, D, i, j, k)]; });
        o += dom_count(K, half);
      }
    return PIC_OK;
  }
  if (kind == PIC_DIAG_POL) {
    double* o = (double*)host_out;
    std::vector<float> buf(L.ncell, 0.0f);
    int dstep = 0;
    HIP_OK(hipMemcpy(&dstep, &c->d_ctr->step, sizeof dstep, hipMemcpyDeviceToHost));
    for (int w = 0; w < 2; ++w)
      for (int q = 0; q < 3; ++q) {
        if (L.lx0 < L.lx1)
          HIP_OK(hipMemcpy(buf.data(), devp(c, w == 0 ? L.o_Q[dstep & 1][q] : L.o_Kp[dstep & 1][q]),
                           sizeof(float) * L.ncell, hipMemcpyDeviceToHost));
        for_domain(K, kHalfE[q], [&](int64_t n, int64_t i, int64_t j, int64_t k) { o[n] = buf[pidx(L, D, i, j, k)]; });
        o += dom_count(K, kHalfE[q]);
      }
    return PIC_OK;
  }
  if (kind == PIC_DIAG_AMP || kind == PIC_DIAG_IMAX) {
    std::vector<float> buf(L.ncell, 0.0f);
    const void* src = kind == PIC_DIAG_AMP ? devp(c, L.o_A) : (const void*)c->d_imax;
    if (src) HIP_OK(hipMemcpy(buf.data(), src, sizeof(float) * L.ncell, hipMemcpyDeviceToHost));
    float* o = (float*)host_out;
    for_domain(K, kNode, [&](int64_t n, int64_t i, int64_t j, int64_t k) { o[n] = buf[pidx(L, D, i, j, k)]; });
    return PIC_OK;
  }
  if (kind == PIC_DIAG_NE_GRID || kind == PIC_DIAG_UE_GRID) {
    HIP_OK(hipMemsetAsync(c->d_grid64, 0, sizeof(double) * L.ncell, s));
    launch_diag_deposit(c->d_inst, D, c->cfg.shape_order, (int)L.capacity, c->d_grid64,
                        kind == PIC_DIAG_NE_GRID ? 1 : 2, s);
    std::vector<double> buf(L.ncell);
    HIP_OK(hipMemcpyAsync(buf.data(), c->d_grid64, sizeof(double) * L.ncell, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    double* o = (double*)host_out;
    std::vector<double> full = buf;
    // fold periodic images are already wrapped by the deposit
    for_domain(K, kNode, [&](int64_t n, int64_t i, int64_t j, int64_t k) { o[n] = full[pidx(L, D, i, j, k)]; });
    return PIC_OK;
  }
  if (kind == PIC_DIAG_PARAMS) {
    pic_params P;
    pic_canonical(&c->cfg, &P);
    for (int m = 0; m < K.nmat; ++m) {
      P.amp_cut[m] = c->tabs[m].acut;
      P.amp_sat[m] = c->tabs[m].asat;
    }
    std::memcpy(host_out, &P, sizeof P);
    return PIC_OK;
  }
  if (kind == PIC_DIAG_SORT) {
    int w[SC_WORDS];
    HIP_OK(hipMemcpy(w, c->d_ctr->sctl, sizeof w, hipMemcpyDeviceToHost));
    double* o = (double*)host_out;
    o[0] = w[SC_NSORTED];
    o[1] = w[SC_NCHUNKS];
    o[2] = w[SC_NDRIFT];
    o[3] = w[SC_NSORTS];
    return PIC_OK;
  }
  if (kind == PIC_DIAG_REGION) {
    // the slot the next step reads, with the tile split the field kernel derives from it
    int x[6], fr = 0;
    unsigned long long td[8 * 32];
    HIP_OK(hipMemcpy(x, c->d_ctr->xext, sizeof x, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(&fr, &c->d_ctr->front, sizeof fr, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(td, c->d_ctr->tiles_done, sizeof td, hipMemcpyDeviceToHost));
    double done = 0.0;
    for (int k = 0; k < 8; ++k) done += (double)td[32 * k];
    int lo = x[2 * (c->step % 3)], hi = x[2 * (c->step % 3) + 1];
    if (L.wx1 > L.wx0) {
      lo = std::min(lo, L.wx0 - G);
      hi = std::max(hi, L.wx1 - 1 - G);
    }
    const int TX = field_tile_x(D, c->tile);
    const int ntx = (int)((L.Px + TX - 1) / TX);
    int nnx = 0;
    if (lo <= hi) {
      const int alo = std::max(0, lo - XNEAR_MARGIN + G);
      const int ahi = std::min((int)L.Px - 1, hi + XNEAR_MARGIN + G);
      if (alo <= ahi) nnx = ahi / TX - alo / TX + 1;
    }
    if (!c->far_skip) nnx = ntx;
    const int rows = c->nb_cell / ntx;
    double* o = (double*)host_out;
    o[0] = lo;
    o[1] = hi;
    o[2] = (double)nnx * rows;
    o[3] = (double)(ntx - nnx) * rows;
    o[4] = fr - G;
    o[5] = done;
    return PIC_OK;
  }
  if (kind == PIC_DIAG_HEALTH) {
    unsigned h = 0;
    int cnt = 0, dstep = 0;
    HIP_OK(hipMemcpy(&h, &c->d_ctr->health, sizeof h, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(&cnt, &c->d_ctr->pcount, sizeof cnt, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(&dstep, &c->d_ctr->step, sizeof dstep, hipMemcpyDeviceToHost));
    double* o = (double*)host_out;
    o[0] = (double)h;
    o[1] = (double)c->latched;
    o[2] = (double)dstep;
    o[3] = (double)cnt;
    return PIC_OK;
  }
  if (kind == PIC_DIAG_TIMERS) {
    harvest_all(c);
    double* o = (double*)host_out;
    for (int ph = 0; ph < 8; ++ph) {
      o[ph] = c->timers[ph];
      o[8 + ph] = c->tcount[ph];
    }
    for (int v = 0; v < 7; ++v) o[16 + v] = c->tune_ms[v];
    o[23] = c->tile;
    o[24] = c->nb_cell;
    o[25] = c->nb_push;
    for (int k = 26; k < 32; ++k) o[k] = 0.0;
    o[26] = c->nvar > 7 ? c->tune_ms[7] : 0.0;   // the z-marching update, where it applies
    o[27] = c->nvar;
    return PIC_OK;
  }
  // ---- SCALARS
  (void)hipGetLastError();
  double* o = (double*)host_out;
  std::memset(o, 0, sizeof(double) * PIC_SC_COUNT);
  HIP_OK(hipMemsetAsync(c->d_ctr->acc, 0, sizeof(c->d_ctr->acc), s));
  launch_diag_particles(c->d_inst, (int)L.capacity, c->d_ctr->acc, s);
  launch_diag_field_energy(c->d_inst, L.ncell, c->d_ctr->acc + 40, s);
  HIP_OK(hipMemsetAsync(c->d_grid64, 0, sizeof(double) * L.ncell, s));
  launch_diag_deposit(c->d_inst, D, c->cfg.shape_order, (int)L.capacity, c->d_grid64, 0, s);
  launch_diag_gauss(c->d_inst, D, c->d_grid64, c->d_ctr->acc + 44, s);
  Ctr h;
  HIP_OK(hipMemcpyAsync(&h, c->d_ctr, sizeof h, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  if (hipGetLastError() != hipSuccess) return PIC_E_DEVICE;
  double ne = 0, np = 0, kee = 0, kep = 0, egap = 0, nev = 0;
  for (int m = 0; m < K.nmat; ++m) {
    ne += h.acc[2 * (2 * m)];
    kee += h.acc[2 * (2 * m) + 1];
    np += h.acc[2 * (2 * m + 1)];
    kep += h.acc[2 * (2 * m + 1) + 1];
    unsigned long long ev = 0;
    for (int x = 0; x < 8; ++x) ev += h.nevents[x * 32 + m];
    nev += (double)ev;
    egap += (double)ev * c->h.kw[2 * m] * K.mats[m].gap_eV * kQE;
  }
  if (c->cfg.preionize_eV > 0) {
    // pre-ionized neutrals count as events of step 0
    nev += (double)L.nneut;
  }
  o[PIC_SC_STEP] = (double)h.step;
  o[PIC_SC_TIME] = h.step * K.dt;
  o[PIC_SC_N_NEUTRAL] = (double)L.nneut - nev;
  o[PIC_SC_N_E] = ne;
  o[PIC_SC_N_POS] = np;
  o[PIC_SC_EVENTS] = nev;
  o[PIC_SC_U_FIELD] = 0.5 * kEPS0 * h.acc[40] * K.vcell;
  o[PIC_SC_KE_E] = kee;
  o[PIC_SC_KE_POS] = kep;
  o[PIC_SC_E_GAP] = egap;
  o[PIC_SC_E_ABS] = kee + kep + egap;
  o[PIC_SC_GAUSS_MAX] = h.acc[44];
  o[PIC_SC_RHO_MAX] = h.acc[45];
  o[PIC_SC_GAUSS_L2] = h.acc[47] > 0 ? std::sqrt(h.acc[46] / h.acc[47]) : 0.0;
  o[PIC_SC_E_IN] = o[PIC_SC_E_OUT] = 0.0;
  for (int x = 0; x < 8; ++x) {
    o[PIC_SC_E_IN] += h.eflux[x * 32];
    o[PIC_SC_E_OUT] += h.eflux[x * 32 + 1];
  }
  o[PIC_SC_HEALTH] = (double)h.health;
  o[PIC_SC_SLOTS] = (double)h.pcount;
  unsigned long long nrec = 0;
  if (c->d_tracks) HIP_OK(hipMemcpy(&nrec, c->d_tracks, sizeof nrec, hipMemcpyDeviceToHost));
  o[PIC_SC_TRACKS_DROPPED] = (double)std::max<int64_t>(0, (int64_t)nrec - c->track_max);
  return PIC_OK;
}

pic_status pic_table_probe_device(pic_ctx* c, int32_t mat, const float* A, int64_t n, float* P_out) {
  if (!c || !A || !P_out || n < 0 || mat < 0 || mat >= c->canon.nmat) return PIC_E_INVAL;
  if (n == 0) return PIC_OK;
  float *dA = nullptr, *dP = nullptr;
  HIP_OK(hipMalloc(&dA, 4 * n));
  if (hipMalloc(&dP, 4 * n) != hipSuccess) {
    (void)hipFree(dA);
    return PIC_E_NOMEM;
  }
  pic_status st = PIC_OK;
  if (hipMemcpy(dA, A, 4 * n, hipMemcpyHostToDevice) != hipSuccess) st = PIC_E_DEVICE;
  if (st == PIC_OK) {
    launch_table_probe((const TabHdr*)devp(c, c->L.o_tab[mat]), dA, dP, n, nullptr);
    if (hipMemcpy(P_out, dP, 4 * n, hipMemcpyDeviceToHost) != hipSuccess) st = PIC_E_DEVICE;
  }
  (void)hipFree(dA);
  (void)hipFree(dP);
  return st;
}

// ------------------------------------------------------------------ batch
pic_status pic_batch_create(pic_ctx* const* members, int32_t n, pic_batch** out) {
  if (!out || n < 0 || (n > 0 && !members)) return PIC_E_INVAL;
  pic_batch* b = new (std::nothrow) pic_batch();
  if (!b) return PIC_E_NOMEM;
  for (int i = 0; i < n; ++i) {
    if (!members[i]) {
      delete b;
      return PIC_E_INVAL;
    }
    b->members.push_back(members[i]);
  }
  if (n > 0) b->stream = members[0]->stream;
  *out = b;
  return PIC_OK;
}

static void batch_drop_graph(pic_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

static void batch_free_classes(pic_batch* b) {
  batch_drop_graph(b);
  for (auto& cl : b->classes) {
    if (cl.d_insts) (void)hipFree(cl.d_insts);
    if (cl.d_off) (void)hipFree(cl.d_off);
    if (cl.d_map) (void)hipFree(cl.d_map);
  }
  b->classes.clear();
}

static pic_status batch_rebuild(pic_batch* b) {
  if (b->stream) (void)hipStreamSynchronize(b->stream); else (void)hipDeviceSynchronize();
  batch_free_classes(b);
  for (pic_ctx* c : b->members) {
    pic_batch::Class* cl = nullptr;
    for (auto& k : b->classes)
      if (k.D == c->canon.D && k.order == c->cfg.shape_order && k.tile == c->tile && k.per == (bool)c->canon.per[1])
        cl = &k;
    if (!cl) {
      b->classes.push_back(pic_batch::Class{});
      cl = &b->classes.back();
      cl->D = c->canon.D;
      cl->order = c->cfg.shape_order;
      cl->tile = c->tile;
      cl->per = c->canon.per[1];
    }
    cl->ms.push_back(c);
    cl->lor = std::max(cl->lor, disp_mode(c->L));
  }
  // persistent push/sort blocks: shared out over the members (every member
  // keeps at least 16; its grid-stride loops cover any particle count)
  const int nmem = (int)b->members.size();
  const int push_share = std::max(16, 8192 / std::max(1, nmem)) / 8 * 8;
  for (auto& cl : b->classes) {
    cl.n = (int)cl.ms.size();
    std::vector<Inst> hi(cl.n);
    std::vector<int> off(4 * (cl.n + 1), 0);
    for (int i = 0; i < cl.n; ++i) {
      hi[i] = cl.ms[i]->h;
      hi[i].step_now = (int)cl.ms[i]->step;
      const int nb[4] = {std::min(cl.ms[i]->nb_push, push_share), cl.ms[i]->nb_cell, cl.ms[i]->nb_win,
                         cl.ms[i]->nb_neut};
      for (int ph = 0; ph < 4; ++ph) off[ph * (cl.n + 1) + i + 1] = off[ph * (cl.n + 1) + i] + nb[ph];
    }
    for (int ph = 0; ph < 4; ++ph) cl.blocks[ph] = off[ph * (cl.n + 1) + cl.n];
    if (cl.n > 65535) return PIC_E_INVAL;
    std::vector<unsigned short> map;
    for (int ph = 0; ph < 4; ++ph) {
      cl.map_off[ph] = (int)map.size();
      for (int i = 0; i < cl.n; ++i)
        map.insert(map.end(), off[ph * (cl.n + 1) + i + 1] - off[ph * (cl.n + 1) + i], (unsigned short)i);
    }
    HIP_OK(hipMalloc(&cl.d_insts, sizeof(Inst) * cl.n));
    HIP_OK(hipMalloc(&cl.d_off, sizeof(int) * off.size()));
    HIP_OK(hipMalloc(&cl.d_map, sizeof(unsigned short) * map.size()));
    HIP_OK(hipMemcpy(cl.d_insts, hi.data(), sizeof(Inst) * cl.n, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(cl.d_off, off.data(), sizeof(int) * off.size(), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(cl.d_map, map.data(), sizeof(unsigned short) * map.size(), hipMemcpyHostToDevice));
  }
  b->expect.clear();
  for (pic_ctx* c : b->members) b->expect.push_back(c->step);
  b->dirty = false;
  return PIC_OK;
}

// Enqueue k batch steps on stream s (the tick decides the sort checks).
static void batch_enqueue(pic_batch* b, int64_t k, hipStream_t s) {
  for (int64_t t = 0; t < k; ++t) {
    const bool sort_due = b->resort > 0 && b->tick++ % b->resort == 0;
    for (auto& cl : b->classes) {
      const int np1 = cl.n + 1;
      Group gp{cl.d_insts, cl.d_off + 0 * np1, cl.n, cl.blocks[0], -1, 0, cl.d_map + cl.map_off[0]};
      Group gc{cl.d_insts, cl.d_off + 1 * np1, cl.n, cl.blocks[1], -1, 1, cl.d_map + cl.map_off[1]};
      gc.lor = cl.lor;
      Group gs{cl.d_insts, cl.d_off + 2 * np1, cl.n, cl.blocks[2], -1, 0, cl.d_map + cl.map_off[2]};
      Group gn{cl.d_insts, cl.d_off + 3 * np1, cl.n, cl.blocks[3], -1, 0, cl.d_map + cl.map_off[3]};
      if (sort_due) launch_sort(gp, gs, cl.D, s);
      launch_push(gp, cl.D, cl.order, cl.per, s);
      launch_fields(gc, cl.D, cl.tile, s);   // far tiles skip the current
      launch_ionize(gn, cl.D, cl.order, s);
      launch_advance(cl.d_insts, cl.n, s);
    }
  }
}

// Capture `period` batch steps, starting at a tick that is a multiple of the
// period (the first of them checks the sort), as a graph; false if capture is
// not possible (the batch then steps eagerly).
static bool batch_capture(pic_batch* b, int period) {
  if (!b->cap && hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) return false;
  const int64_t tick = b->tick;
  if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
  batch_enqueue(b, period, b->cap);
  b->tick = tick;   // nothing ran: the capture only recorded the launches
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(b->cap, &g) != hipSuccess || !g) return false;
  b->graph = g;
  if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    batch_drop_graph(b);
    return false;
  }
  return true;
}

pic_status pic_batch_step(pic_batch* b, int64_t nsteps) {
  if (!b || nsteps < 0) return PIC_E_INVAL;
  for (pic_ctx* c : b->members)
    if (c->latched != PIC_OK || c->imax_every > 0 || c->track_every > 0) return PIC_E_STATE;
  // a member stepped, restored or given a state outside the batch: its step
  // index in the batch's parameter blocks is stale
  for (size_t i = 0; !b->dirty && i < b->members.size(); ++i)
    if (i >= b->expect.size() || b->members[i]->step != b->expect[i]) b->dirty = true;
  if (b->dirty) {
    pic_status st = batch_rebuild(b);
    if (st != PIC_OK) return st;
  }
  hipStream_t s = b->stream;
  (void)hipGetLastError();
  int64_t left = nsteps;
  const int period = b->resort > 0 ? b->resort : 8;
  if (b->graph_on && !b->classes.empty() && period <= 64 && left >= period) {
    // eager steps up to the next multiple of the sort period, then replays
    const int64_t lead = std::min<int64_t>(left, (period - b->tick % period) % period);
    batch_enqueue(b, lead, s);
    left -= lead;
    if (left >= period && !b->exec && !batch_capture(b, period)) {
      (void)hipGetLastError();
      b->graph_on = 0;   // capture unavailable: step eagerly from now on
    }
    while (b->exec && left >= period) {
      if (hipGraphLaunch(b->exec, s) != hipSuccess) return PIC_E_DEVICE;
      b->tick += period;
      left -= period;
      ++b->replays;
    }
  }
  batch_enqueue(b, left, s);
  for (pic_ctx* c : b->members) c->step += nsteps;
  for (auto& e : b->expect) e += nsteps;
  if (hipGetLastError() != hipSuccess) return PIC_E_DEVICE;
  return PIC_OK;
}

pic_status pic_batch_set_graph(pic_batch* b, int32_t on) {
  if (!b) return PIC_E_INVAL;
  b->graph_on = on ? 1 : 0;
  return PIC_OK;
}

int64_t pic_batch_graph_replays(const pic_batch* b) { return b ? b->replays : 0; }

pic_status pic_batch_add(pic_batch* b, pic_ctx* c) {
  if (!b || !c || c->canon.collide || c->canon.impact) return PIC_E_INVAL;
  for (pic_ctx* m : b->members)
    if (m == c) return PIC_E_INVAL;
  if (b->members.empty()) b->stream = c->stream;
  b->members.push_back(c);
  b->dirty = true;
  return PIC_OK;
}

pic_status pic_batch_remove(pic_batch* b, pic_ctx* c) {
  if (!b || !c) return PIC_E_INVAL;
  auto it = std::find(b->members.begin(), b->members.end(), c);
  if (it == b->members.end()) return PIC_E_INVAL;
  b->members.erase(it);
  b->dirty = true;
  return PIC_OK;
}

void pic_batch_destroy(pic_batch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream); else (void)hipDeviceSynchronize();
  batch_free_classes(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}

}  // extern "C"
