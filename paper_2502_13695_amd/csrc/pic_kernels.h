// Device kernels of the PIC hot path (gfx950).  Every kernel advances a group
// of independent instances in one launch: block b belongs to the instance i
// with off[i] <= b < off[i+1] (a single run is a group of one).
#pragma once

#include "pic_common.h"

namespace pic {

struct Group {
  const Inst* insts;   // device array of instance parameter blocks
  const int* off;      // device prefix offsets of blocks per instance (n + 1)
  int n;               // instances
  int blocks;          // total blocks
  int step;            // step index of a single run; -1: each instance's device counter
  // field update: 0 every tile reads its current; 1 far tiles skip the current
  // and far tiles beyond the field front are not updated; 2 far tiles skip the
  // current but every tile is updated (the in-run timing of the tile shapes)
  int part = 0;
  // batches: the instance of every block (one load instead of a binary search
  // over `off`); null for a single run
  const unsigned short* map = nullptr;
  // a single run's field front and charged-region slots, read directly so
  // they load alongside the instance block instead of after it; null in
  // batches (each instance's own, through its parameter block)
  int* front = nullptr;
  const int* xext = nullptr;
  // host copy of a single run's parameter block: the field launch passes it
  // by value, so its fields load from the kernel arguments
  const Inst* host = nullptr;
  // dispersive media in the field update: 0 none; 1 Lorentz oscillators; 2
  // Kerr terms too (some instance has them).  Each a kernel variant of its
  // own, so runs without them keep their registers.
  int lor = 0;
};

constexpr int TPB = 256;

// Optional events stamped by the dispatch itself (start of the phase's first
// kernel, end of its last): kernel execution time, without the gap between a
// separately recorded event and the dispatch that follows it.
struct Stamp {
  hipEvent_t start = nullptr, stop = nullptr;
};

// phase launchers (enqueue on `s`); D = 1..3, order = 1..2
// per: periodic transverse axes (D >= 2)
// Blocks of the push grid: as many as are resident at once on this GPU (a
// multiple of 8; the blocks take their work from queues).  0 on error.
int push_grid(int D);
void launch_push(const Group& g, int D, int order, bool per, hipStream_t s, Stamp st = {});
// tile sort of the charged particles (gp: the push grid; gscan: one block per
// instance); each instance decides on the device whether a sort is due
void launch_sort(const Group& gp, const Group& gscan, int D, hipStream_t s, Stamp st = {});
void launch_fields(const Group& g, int D, int variant, hipStream_t s, Stamp st = {});
void launch_ionize(const Group& g, int D, int order, hipStream_t s, Stamp st = {});
// suffix maxima of the amplitude window (a single run, after the field update
// of a step whose slot is nwin - 1)
void launch_win_rebuild(const Inst& I, int64_t wsz, hipStream_t s, hipEvent_t stop = nullptr);
void launch_advance(Inst* insts, int n, hipStream_t s);   // batch: step counters + 1

// Binary collisions (a single run): device work arrays over the box cells
// (ncell = nx ny nz) and the charged slots.
constexpr int COL_SCAN_B = 1024;   // cells per block of the cell scan
struct ColBufs {
  int* cnt;       // ncell + 1: particles per cell, then (scanned) each cell's first index
  int* fill;      // ncell: particles placed per cell
  int* bsum;      // col_scan_blocks(ncell + 1) + 1: block sums of the scan
  int* idx;       // capacity: slots ordered by cell
  uint64_t* key;  // capacity: order key of each entry of idx (kind, then the pairing key)
  // the cells that take part (collisions: at least two particles; impact
  // ionization: at least one): listed per block of COL_SCAN_B cells at the
  // front of that block's COL_SCAN_B entries of active, their number per
  // block in bact (then scanned: the blocks' offsets, the total last), then
  // gathered into list
  int* active;    // col_scan_blocks(ncell + 1) * COL_SCAN_B
  int* bact;      // col_scan_blocks(ncell + 1) + 1
  int* list;      // capacity
  int ncell;
  double dt;      // time step [s]
  int nk;         // particle kinds of the run (2 per material)
  int collide;    // binary collisions
  int impact;     // impact ionization
  // impact ionization: per material the rate constant [1/s], threshold [J]
  // and gap [J]; per cell x index the rank among the material x cells (-1:
  // none) and their count, so cell (i, j, k) holds neutrals from
  // ((j + ny k) nmx + mrank[i]) ppc on
  double imp_P[MAXMAT], imp_th[MAXMAT], gap[MAXMAT];
  const int* mrank;
  int nmx;
};
int col_scan_blocks(int n);
// collisions and impact ionization of the step whose index after
// photoionization is `step` (the state after the step's push and
// photoionization), on stream s
void launch_collide(const Inst& I, const ColBufs& b, int step, hipStream_t s, Stamp st = {});
int field_tiles(int D, int variant, int Px, int Py, int Pz);   // blocks of the field launch
// field tile shapes of a run: the tiled shapes, plus the z-marching update in
// 3D when y and z are periodic
int field_tile_variants(int D, bool periodic_yz);
int field_tile_x(int D, int variant);                          // owned x extent of a field tile

// one-instance setup and diagnostics
void launch_init_neutrals_d(const Inst* d, int64_t nneut, int D, hipStream_t s);
void launch_preionize_d(const Inst* d, int64_t nneut, int D, const float* sig_e, const float* sig_p,
                        hipStream_t s);
// energy histogram of the charged particles (per kind, over caller edges)
struct SpecArgs {
  int nkinds, nedges;      // rows; increasing edges (columns = nedges + 1)
  int x_lo, x_hi;          // x cells counted (x_hi <= x_lo: every cell)
  int lds;                 // counts fit in LDS beside the edges (spec_lds_counts)
  double mc2_eV[MAXKIND];  // rest energy per kind [eV]
};
// LDS per block: the edges (8 B each) and, when they fit in 64 KB with them,
// the counts (4 B per kind and column)
inline bool spec_lds_counts(int nkinds, int nedges) {
  return 8u * nedges + 4u * nkinds * (nedges + 1) <= 65536u - 1024u;
}
void launch_spectrum(const Inst* d, int D, int capacity, const SpecArgs& a, const double* edges,
                     unsigned long long* out, hipStream_t s);
// running maximum of the node |E|^2 over the domain nodes
struct ImaxArgs {
  const float *E0, *E1, *E2;   // E after the step's field update (padded layout)
  int64_t nodes;               // domain nodes: mx * my * mz
  int mx, my;
  int D, nx, ny, nz, per_y, per_z;
  int Gy, Gz;                  // guard layers of y and z (x: G)
  int64_t sy, sz;
};
void launch_imax(const ImaxArgs& a, float* imax, hipStream_t s);
// one record of a sampled particle (the layout of pic_track)
struct TrackRec {
  uint32_t id;
  int32_t kind, step;
  int32_t cell[3];
  float off[3];
  int32_t pad;
};
void launch_tracks(const Inst* d, int D, int capacity, uint32_t thr, int step, TrackRec* rec,
                   unsigned long long* n, int64_t max_records, hipStream_t s);
void launch_diag_particles(const Inst* d, int capacity, double* acc, hipStream_t s);
void launch_diag_field_energy(const Inst* d, int64_t ncell, double* acc, hipStream_t s);
void launch_diag_deposit(const Inst* d, int D, int order, int capacity, double* grid, int what,
                         hipStream_t s);
void launch_diag_gauss(const Inst* d, int D, const double* rho, double* acc, hipStream_t s);
void launch_table_probe(const TabHdr* tab, const float* A, float* P, int64_t n, hipStream_t s);

}  // namespace pic
