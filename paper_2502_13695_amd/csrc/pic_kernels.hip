// Device kernels of the MI355X laser-dielectric PIC hot path.
//
// Three launches per step (state E^n, b^n = cB^n in field set n & 1, particles
// x^n with u^{n-1/2}):
//   push      gather E^n, b^n with the particle shape, relativistic Boris,
//             move, Esirkepov deposit of J^{n+1/2} (global FP32 atomics)
//   fields    one LDS tile per block: b^{n+1/2} = b^n - (1/2) C curl E^n,
//             E^{n+1} = E^n + (1/eps_r)(C curl b^{n+1/2} - dt J / eps0), the
//             first-order outflow (Mur) chain on the faces with the laser
//             injected at x_min, b^{n+1} = b^{n+1/2} - (1/2) C curl E^{n+1}
//             (written to the other field set), J cleared, node |E^{n+1}| into
//             the one-cycle window with its exact sliding maximum (van Herk /
//             Gil-Werman blocks) giving the amplitude A (Sec. 2.1)
//   ionize    per alive neutral: A at the neutral (shape gather), P from the
//             FP32 Keldysh table (Sec. 2.1), Philox draw, electron and
//             positive-carrier birth (Sec. 2.1, 3.2); the last block advances
//             the step counter
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <type_traits>

#include "pic_kernels.h"

namespace pic {

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ int find_inst(const Group& g) {
  if (g.map) return g.map[blockIdx.x];
  const int b = blockIdx.x;
  int lo = 0, hi = g.n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (g.off[mid] <= b) lo = mid; else hi = mid;
  }
  return lo;
}

// Instance of this block, the block's index within the instance's range and
// the range's length.  A single run (one instance, offsets {0, blocks}) needs
// no memory access for this.
struct Slot {
  int ii, bk, nbk;
};
__device__ __forceinline__ Slot block_slot(const Group& g) {
  if (g.n == 1) return {0, (int)blockIdx.x, g.blocks};
  const int ii = find_inst(g);
  return {ii, (int)blockIdx.x - g.off[ii], g.off[ii + 1] - g.off[ii]};
}

// The parameter block of a kernel launched either for a single run (the
// block itself passed by value) or for a batch (an array indexed per block).
struct NoInst {};
__device__ __forceinline__ const Inst& inst_of(const Group&, int, const Inst& one) { return one; }
// Batches: no kernel writes the array, so it is read through the constant
// address space (its fields are not reloaded after every other store).
using CInst = const __attribute__((address_space(4))) Inst;
__device__ __forceinline__ CInst& inst_of(const Group& g, int ii, NoInst) { return *(CInst*)(g.insts + ii); }

// Workgroups are dispatched to the 8 XCDs (each with its own L2) round robin,
// block b going to XCD b mod 8.  Work index of block b of nb such that every
// XCD walks a contiguous range of the work (neighbouring tiles share halo
// lines in one L2).  A bijection of [0, nb).
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7, s = b >> 3;
  return x * q + (x < r ? x : r) + s;
}

__device__ __forceinline__ int wrapi(int j, int n, int per) {
  if (!per) return j;
  return j < 0 ? j + n : (j >= n ? j - n : j);
}

// Global-memory views of device pointers: loads, stores and atomics through
// them compile to global_* instructions (scalar base + 32-bit offset) instead
// of flat ones, which would also wait on LDS traffic.
template <class T>
using gmem = __attribute__((address_space(1))) T;
template <class T>
__device__ __forceinline__ gmem<T>* gp(T* p) {
  return (gmem<T>*)p;
}
template <class T>
__device__ __forceinline__ const gmem<T>* gp(const T* p) {
  return (const gmem<T>*)p;
}
// A pointer every lane holds the same value of, made visibly wave-uniform (kept
// in scalar registers: loads through it use a scalar base + 32-bit offset).
template <class T>
__device__ __forceinline__ T* uniform(T* p) {
  const unsigned long long v = (unsigned long long)p;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return (T*)(((unsigned long long)hi << 32) | lo);
}

// Element i of an array through a 32-bit byte offset from a wave-uniform
// base: the scalar-base addressing form, one VALU shift per offset shared by
// every array indexed with it (grids hold fewer than 2^30 points).
template <class T>
__device__ __forceinline__ const gmem<T>& at(const gmem<T>* b, unsigned i) {
  return *(const gmem<T>*)((const gmem<char>*)b + i * (unsigned)sizeof(T));
}
template <class T>
__device__ __forceinline__ gmem<T>& at(gmem<T>* b, unsigned i) {
  return *(gmem<T>*)((gmem<char>*)b + i * (unsigned)sizeof(T));
}

// shape weights on the integer grid for a particle at cell c + offset t
// (t in [0,1)); half = 1 for a half-integer staggered component.
// Returns the first grid index; weights w[0..ORDER].
template <int ORDER>
__device__ __forceinline__ int shape(int c, float t, int half, float* w) {
  if (ORDER == 2) {
    if (half) {
      const float xi = t - 0.5f;
      w[0] = 0.5f * (0.5f - xi) * (0.5f - xi);
      w[1] = 0.75f - xi * xi;
      w[2] = 0.5f * (0.5f + xi) * (0.5f + xi);
      return c - 1;
    }
    const int up = t >= 0.5f;
    const float xi = t - (float)up;
    w[0] = 0.5f * (0.5f - xi) * (0.5f - xi);
    w[1] = 0.75f - xi * xi;
    w[2] = 0.5f * (0.5f + xi) * (0.5f + xi);
    return c + up - 1;
  } else {
    if (half) {
      if (t >= 0.5f) {
        const float f = t - 0.5f;
        w[0] = 1.0f - f;
        w[1] = f;
        return c;
      }
      const float f = t + 0.5f;
      w[0] = 1.0f - f;
      w[1] = f;
      return c - 1;
    }
    w[0] = 1.0f - t;
    w[1] = t;
    return c;
  }
}

// ------------------------------------------------------------ particle push
// Stencil of one axis: padded-array offsets (already multiplied by stride and
// wrapped on periodic axes) and weights, node- and half-staggered.
template <int ORDER>
struct Axis {
  int on[ORDER + 1], oh[ORDER + 1];
  float wn[ORDER + 1], wh[ORDER + 1];
};

template <int ORDER>
__device__ __forceinline__ void make_axis(Axis<ORDER>& a, int c, float t, int n, int per, int goff,
                                          int stride) {
  const int bn = shape<ORDER>(c, t, 0, a.wn);
  const int bh = shape<ORDER>(c, t, 1, a.wh);
#pragma unroll
  for (int q = 0; q <= ORDER; ++q) {
    a.on[q] = stride * (wrapi(bn + q, n, per) + goff);
    a.oh[q] = stride * (wrapi(bh + q, n, per) + goff);
  }
}

template <int D, int ORDER>
__device__ __forceinline__ float gather(const float* __restrict__ Fp, const Axis<ORDER>& X,
                                        const Axis<ORDER>& Y, const Axis<ORDER>& Z, int hx, int hy,
                                        int hz) {
  constexpr int SY = D >= 2 ? ORDER + 1 : 1;
  constexpr int SZ = D >= 3 ? ORDER + 1 : 1;
  constexpr int SX = ORDER + 1;
  const gmem<float>* __restrict__ F = gp(Fp);
  // all loads first (independent, in flight together), then the weighted sum;
  // x is never periodic, so the x nodes are consecutive
  const int ox = hx ? X.oh[0] : X.on[0];
  float v[SZ][SY][SX];
#pragma unroll
  for (int c = 0; c < SZ; ++c) {
    const int oz = D >= 3 ? (hz ? Z.oh[c] : Z.on[c]) : 0;
#pragma unroll
    for (int b = 0; b < SY; ++b) {
      const int oy = D >= 2 ? (hy ? Y.oh[b] : Y.on[b]) : 0;
      const gmem<float>* __restrict__ r = F + (ox + oy + oz);
#pragma unroll
      for (int a = 0; a < SX; ++a) v[c][b][a] = r[a];
    }
  }
  float acc = 0.0f;
#pragma unroll
  for (int c = 0; c < SZ; ++c) {
    const float wz = D >= 3 ? (hz ? Z.wh[c] : Z.wn[c]) : 1.0f;
#pragma unroll
    for (int b = 0; b < SY; ++b) {
      const float wy = D >= 2 ? (hy ? Y.wh[b] : Y.wn[b]) : 1.0f;
      float row = 0.0f;
#pragma unroll
      for (int a = 0; a < SX; ++a) row += (hx ? X.wh[a] : X.wn[a]) * v[c][b][a];
      acc += wz * wy * row;
    }
  }
  return acc;
}

// Esirkepov arrays along one axis, compacted to the W = ORDER + 2 nodes a
// move of at most one cell can touch, from `org` = the lower of the start and
// end shape bases: S0 = start weights, DS = end - start weights.  A move that
// keeps its shape base leaves node W - 1 zero.
//
// DS is formed from the two offsets (32-bit fractions) in factored form, with
// the small differences taken on the integers: subtracting two sets of
// rounded weights would leave a few 1e-8 on every node whatever the move, a
// relative error of 1e-5 on the current of a particle that moves 1e-3 cells
// per step (a thermal plasma).  Quadratic shape, xi0 and xi1 = the offsets
// from the centres of their own stencils (xi 2^32 = o read as a signed
// integer):
//   same base:   d = xi1 - xi0, s = xi0 + xi1;
//                DS = (-d (1 - s) / 2, -d s, d (1 + s) / 2)
//   base up:     a = xi0 - 1/2 <= 0, e = xi1 + 1/2 >= 0;
//                DS = (-a^2/2, (a - e) + a^2 + e^2/2, (e - a) - e^2 - a^2/2, e^2/2)
//   base down:   the mirror image (a = -xi0 - 1/2, e = 1/2 - xi1, reversed).
// Linear shape: d = t1 - t0 on a kept cell, else 1 - t first.  A difference
// below 1/4 is read off the integers (exact up to its FP32 rounding, no wrap
// below 1/2); a larger one loses nothing in FP32.
__device__ __forceinline__ float fix_small(uint32_t v, float approx) {
  return fabsf(approx) < 0.25f ? (float)(int32_t)v * 0x1p-32f : approx;
}

template <int ORDER>
struct Esk {
  static constexpr int W = ORDER + 2;
  float S0[W], DS[W];
  int org;
  int moved;   // the shape base changed along this axis
};

template <int ORDER>
__device__ __forceinline__ void esk_axis(Esk<ORDER>& e, int c0, uint32_t o0, int c1, uint32_t o1) {
  if (ORDER == 2) {
    const int up0 = o0 >= 0x80000000u, up1 = o1 >= 0x80000000u;
    const float xi0 = (float)(int32_t)o0 * 0x1p-32f, xi1 = (float)(int32_t)o1 * 0x1p-32f;
    const float w0 = 0.5f * (0.5f - xi0) * (0.5f - xi0);
    const float w1 = 0.75f - xi0 * xi0;
    const float w2 = 0.5f * (0.5f + xi0) * (0.5f + xi0);
    const int b0 = c0 + up0 - 1;
    const int sh = (c1 + up1 - 1) - b0;   // -1, 0, 1
    e.moved = sh != 0;
    if (sh < 0) {
      const float a = -fix_small(o0 + 0x80000000u, 0.5f + xi0);
      const float f = -fix_small(o1 - 0x80000000u, xi1 - 0.5f);
      e.org = b0 - 1;
      e.S0[0] = 0.0f;
      e.S0[1] = w0;
      e.S0[2] = w1;
      e.S0[3] = w2;
      e.DS[0] = 0.5f * f * f;
      e.DS[1] = (f - a) - f * f - 0.5f * a * a;
      e.DS[2] = (a - f) + a * a + 0.5f * f * f;
      e.DS[3] = -0.5f * a * a;
    } else {
      e.org = b0;
      e.S0[0] = w0;
      e.S0[1] = w1;
      e.S0[2] = w2;
      e.S0[3] = 0.0f;
      if (sh > 0) {
        const float a = fix_small(o0 - 0x80000000u, xi0 - 0.5f);
        const float f = fix_small(o1 + 0x80000000u, xi1 + 0.5f);
        e.DS[0] = -0.5f * a * a;
        e.DS[1] = (a - f) + a * a + 0.5f * f * f;
        e.DS[2] = (f - a) - f * f - 0.5f * a * a;
        e.DS[3] = 0.5f * f * f;
      } else {
        const float d = fix_small(o1 - o0, xi1 - xi0), sm = xi0 + xi1;
        e.DS[0] = -0.5f * d * (1.0f - sm);
        e.DS[1] = -d * sm;
        e.DS[2] = 0.5f * d * (1.0f + sm);
        e.DS[3] = 0.0f;
      }
    }
  } else {
    const float t0 = off_lo(o0), t1 = off_lo(o1);
    const int sh = c1 - c0;
    e.moved = sh != 0;
    if (sh < 0) {
      e.org = c0 - 1;
      e.S0[0] = 0.0f;
      e.S0[1] = 1.0f - t0;
      e.S0[2] = t0;
      const float r1 = fix_small(0u - o1, 1.0f - t1);   // 1 - t1
      const float tt0 = fix_small(o0, t0);
      e.DS[0] = r1;
      e.DS[1] = tt0 - r1;
      e.DS[2] = -tt0;
    } else {
      e.org = c0;
      const float r0 = fix_small(0u - o0, 1.0f - t0);   // 1 - t0 (o0 > 0 when small)
      e.S0[0] = 1.0f - t0;
      e.S0[1] = t0;
      e.S0[2] = 0.0f;
      if (sh > 0) {
        const float tt1 = fix_small(o1, t1);
        e.DS[0] = -r0;
        e.DS[1] = r0 - tt1;
        e.DS[2] = tt1;
      } else {
        const float d = fix_small(o1 - o0, t1 - t0);
        e.DS[0] = -d;
        e.DS[1] = d;
        e.DS[2] = 0.0f;
      }
    }
  }
}

// Nodes visited along an axis: W if any lane of the wave changed its shape
// base along it, else W - 1.  Wave-uniform, so the unrolled deposit loops
// below branch on scalars; a lane that did not move adds zeros (or the
// rounding residue of its vanishing cumulative sum) on the extra node.
template <int ORDER>
__device__ __forceinline__ int wave_extent(int moved) {
  return __any(moved) ? ORDER + 2 : ORDER + 1;
}

// Current sinks.  x/y/z map an (unwrapped) node index to an offset; coef()
// prepares a particle factor and wt() a node-pair weight in the sink's
// arithmetic, put() adds coef x wt to component `comp` at offset o.
template <bool PY, bool PZ>
struct GSink {   // the padded HBM arrays, FP32 atomics, periodic wrap
  float* J0;
  float* J1;
  float* J2;
  int ny, nz, sy, sz, Gy, Gz;
  using C = float;
  __device__ __forceinline__ int x(int i) const { return i + G; }
  __device__ __forceinline__ int y(int j) const { return sy * (wrapi(j, ny, PY) + Gy); }
  __device__ __forceinline__ int z(int k) const { return sz * (wrapi(k, nz, PZ) + Gz); }
  __device__ __forceinline__ float coef(float c) const { return c; }
  __device__ __forceinline__ float wt(float w) const { return w; }
  __device__ __forceinline__ void put(int comp, int o, float c, float w) const {
    gmem<float>* J = gp(comp == 0 ? J0 : comp == 1 ? J1 : J2);
    __hip_atomic_fetch_add(J + (unsigned)o, c * w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
};

template <int D>
struct PWin {   // LDS deposit window of a particle tile
  static constexpr int X = ptile_ext(D, 0) + PT_PAD;
  static constexpr int Y = D >= 2 ? ptile_ext(D, 1) + PT_PAD : 1;
  static constexpr int Z = D >= 3 ? ptile_ext(D, 2) + PT_PAD : 1;
  static constexpr int N = X * Y * Z;
};

// The block's LDS window, origin (x0, y0, z0) in unwrapped nodes, 64-bit
// fixed point (integer LDS atomics run at full rate; FP32 LDS atomics do not on
// gfx950): a contribution c w (c = charge factor x scale, w = shape weight) is
// added as round(c w) through an FP64 fma with 1.5 2^52, which leaves the
// integer in the low mantissa bits; the constant's low word is zero, so
// removing it touches the high word only.  Sums are exact and do not depend on
// the order of the atomics.
template <int D>
struct LSink {
  unsigned long long* s;
  int x0, y0, z0;
  double scale;
  using C = double;
  __device__ __forceinline__ int x(int i) const { return i - x0; }
  __device__ __forceinline__ int y(int j) const { return (j - y0) * PWin<D>::X; }
  __device__ __forceinline__ int z(int k) const { return (k - z0) * (PWin<D>::X * PWin<D>::Y); }
  __device__ __forceinline__ double coef(float c) const { return (double)c * scale; }
  __device__ __forceinline__ double wt(float w) const { return (double)w; }
  __device__ __forceinline__ void put(int comp, int o, double c, double w) const {
    const double d = fma(w, c, 6755399441055744.0);
    atomicAdd(s + comp * PWin<D>::N + o, (unsigned long long)__double_as_longlong(d) - 0x4338000000000000ull);
  }
};

// Esirkepov deposit of dt J^{n+1/2} / eps0 for one particle.  Components along
// present axes are -q dx times the cumulative sum of W along their axis, and
// Esirkepov's W_x(i, j, k) = DS_x(i) wb(j, k) with the path-averaged transverse
// weight wb = S0_y S0_z + DS_y S0_z / 2 + S0_y DS_z / 2 + DS_y DS_z / 3, so
// J_x(i, j, k) = (-q dx CS_x(i)) wb(j, k), CS_x the cumulative sum of DS_x;
// wb factors as S0_z (S0_y + DS_y/2) + DS_z (S0_y/2 + DS_y/3).  Components along
// absent axes take q v times the path-averaged shape.
template <int D, int ORDER, class S>
__device__ __forceinline__ void deposit(const S& s, const Esk<ORDER>& ex, const Esk<ORDER>& ey,
                                        const Esk<ORDER>& ez, float qx, float qy, float qz, float vy,
                                        float vz) {
  using CT = typename S::C;
  constexpr int W = ORDER + 2;
  constexpr int WY = D >= 2 ? W : 1;
  constexpr int WZ = D >= 3 ? W : 1;
  const int nx = wave_extent<ORDER>(ex.moved);
  const int ny = D >= 2 ? wave_extent<ORDER>(ey.moved) : 1;
  const int nz = D >= 3 ? wave_extent<ORDER>(ez.moved) : 1;
  constexpr float third = 1.0f / 3.0f;
  // per-axis factors: A = S0 + DS/2, B = S0/2 + DS/3 (absent axes: S0 = 1, DS = 0)
  float Ax[W], Bx[W], Ay[WY], By[WY];
  CT cx[W - 1], cy[W - 1], cz[W - 1];
  {
    float cs = 0.0f;
#pragma unroll
    for (int a = 0; a < W; ++a) {
      Ax[a] = ex.S0[a] + 0.5f * ex.DS[a];
      Bx[a] = 0.5f * ex.S0[a] + third * ex.DS[a];
      if (a < W - 1) {
        cs += ex.DS[a];
        cx[a] = s.coef(-qx * cs);
      }
    }
  }
#pragma unroll
  for (int b = 0; b < WY; ++b) {
    Ay[b] = D >= 2 ? ey.S0[b] + 0.5f * ey.DS[b] : 1.0f;
    By[b] = D >= 2 ? 0.5f * ey.S0[b] + third * ey.DS[b] : 0.5f;
  }
  if (D >= 2) {
    float cs = 0.0f;
#pragma unroll
    for (int b = 0; b < W - 1; ++b) {
      cs += ey.DS[b];
      cy[b] = s.coef(-qy * cs);
    }
  }
  if (D >= 3) {
    float cs = 0.0f;
#pragma unroll
    for (int c = 0; c < W - 1; ++c) {
      cs += ez.DS[c];
      cz[c] = s.coef(-qz * cs);
    }
  }
  // offsets of the nodes along each axis
  int ox[W], oy[WY], oz[WZ];
#pragma unroll
  for (int a = 0; a < W; ++a) ox[a] = s.x(ex.org + a);
#pragma unroll
  for (int b = 0; b < WY; ++b) oy[b] = D >= 2 ? s.y(ey.org + b) : 0;
#pragma unroll
  for (int c = 0; c < WZ; ++c) oz[c] = D >= 3 ? s.z(ez.org + c) : 0;
  // Jx over (j, k)
#pragma unroll
  for (int c = 0; c < WZ; ++c) {
    if (c >= nz) break;
    const float s0z = D >= 3 ? ez.S0[c] : 1.0f, dsz = D >= 3 ? ez.DS[c] : 0.0f;
#pragma unroll
    for (int b = 0; b < WY; ++b) {
      if (b >= ny) break;
      const CT w = s.wt(s0z * Ay[b] + dsz * By[b]);
#pragma unroll
      for (int a = 0; a < W - 1; ++a) {
        if (a >= nx - 1) break;
        s.put(0, ox[a] + oy[b] + oz[c], cx[a], w);
      }
    }
  }
  // Jy over (i, k)
  if (D >= 2) {
#pragma unroll
    for (int c = 0; c < WZ; ++c) {
      if (c >= nz) break;
      const float s0z = D >= 3 ? ez.S0[c] : 1.0f, dsz = D >= 3 ? ez.DS[c] : 0.0f;
#pragma unroll
      for (int a = 0; a < W; ++a) {
        if (a >= nx) break;
        const CT w = s.wt(s0z * Ax[a] + dsz * Bx[a]);
#pragma unroll
        for (int b = 0; b < W - 1; ++b) {
          if (b >= ny - 1) break;
          s.put(1, ox[a] + oy[b] + oz[c], cy[b], w);
        }
      }
    }
  } else {
    const CT c1 = s.coef(qy * vy);
#pragma unroll
    for (int a = 0; a < W; ++a) {
      if (a >= nx) break;
      s.put(1, ox[a], c1, s.wt(Ax[a]));
    }
  }
  // Jz over (i, j)
  if (D >= 3) {
#pragma unroll
    for (int b = 0; b < WY; ++b) {
      if (b >= ny) break;
#pragma unroll
      for (int a = 0; a < W; ++a) {
        if (a >= nx) break;
        const CT w = s.wt(ey.S0[b] * Ax[a] + ey.DS[b] * Bx[a]);
#pragma unroll
        for (int c = 0; c < W - 1; ++c) {
          if (c >= nz - 1) break;
          s.put(2, ox[a] + oy[b] + oz[c], cz[c], w);
        }
      }
    }
  } else {
    const CT c2 = s.coef(qz * vz);
#pragma unroll
    for (int b = 0; b < WY; ++b) {
      if (b >= ny) break;
      const float s0y = D >= 2 ? ey.S0[b] : 1.0f, dsy = D >= 2 ? ey.DS[b] : 0.0f;
#pragma unroll
      for (int a = 0; a < W; ++a) {
        if (a >= nx) break;
        s.put(2, ox[a] + oy[b], c2, s.wt(s0y * Ax[a] + dsy * Bx[a]));
      }
    }
  }
}

// Field sets read by the push of one step.
struct PushFields {
  const float* __restrict__ E0;
  const float* __restrict__ E1;
  const float* __restrict__ E2;
  const float* __restrict__ B0;
  const float* __restrict__ B1;
  const float* __restrict__ B2;
};

// Field window of a particle tile staged in LDS: the gather stencil of a
// particle starting in cell c spans nodes c - 1 .. c + 2 (both staggerings,
// order <= 2), so a tile of T cells needs T + 3 nodes per present axis.
template <int D>
struct FWin {
  static constexpr int X = ptile_ext(D, 0) + 3;
  static constexpr int Y = D >= 2 ? ptile_ext(D, 1) + 3 : 1;
  static constexpr int Z = D >= 3 ? ptile_ext(D, 2) + 3 : 1;
  static constexpr int N = X * Y * Z;
};

// Threads per push block.  In 3D the two LDS windows (85 KB) take most of a
// CU's LDS, so one block of 16 waves per CU shares them.
__host__ __device__ constexpr int push_tpb(int D) { return D == 3 ? 512 : 256; }

template <int ORDER>
__device__ __forceinline__ void make_axis_l(Axis<ORDER>& a, int c, float t, int origin, int stride) {
  const int bn = shape<ORDER>(c, t, 0, a.wn);
  const int bh = shape<ORDER>(c, t, 1, a.wh);
#pragma unroll
  for (int q = 0; q <= ORDER; ++q) {
    a.on[q] = stride * (bn + q - origin);
    a.oh[q] = stride * (bh + q - origin);
  }
}

template <int D, int ORDER>
__device__ __forceinline__ float gather_l(const float* __restrict__ S, const Axis<ORDER>& X,
                                          const Axis<ORDER>& Y, const Axis<ORDER>& Z, int hx, int hy,
                                          int hz) {
  // the window's rows are consecutive nodes, so only the first node of each
  // axis is needed: every other stencil point is a constant offset from it
  constexpr int SY = D >= 2 ? ORDER + 1 : 1;
  constexpr int SZ = D >= 3 ? ORDER + 1 : 1;
  constexpr int SX = ORDER + 1;
  constexpr int LY = FWin<D>::X, LZ = FWin<D>::X * FWin<D>::Y;
  const float* __restrict__ r0 = S + (hx ? X.oh[0] : X.on[0]) + (D >= 2 ? (hy ? Y.oh[0] : Y.on[0]) : 0) +
                                 (D >= 3 ? (hz ? Z.oh[0] : Z.on[0]) : 0);
  float acc = 0.0f;
#pragma unroll
  for (int c = 0; c < SZ; ++c) {
    const float wz = D >= 3 ? (hz ? Z.wh[c] : Z.wn[c]) : 1.0f;
#pragma unroll
    for (int b = 0; b < SY; ++b) {
      const float wy = D >= 2 ? (hy ? Y.wh[b] : Y.wn[b]) : 1.0f;
      const float* r = r0 + b * LY + c * LZ;
      float row = 0.0f;
#pragma unroll
      for (int a = 0; a < SX; ++a) row += (hx ? X.wh[a] : X.wn[a]) * r[a];
      acc += wz * wy * row;
    }
  }
  return acc;
}

// Boris, move, deposit and write-back of one charged particle.  LOCAL: the
// particle started inside the block's tile -- fields from the LDS window
// (origin fx0, fy0, fz0), current into the LDS sink; else HBM for both.  PY,
// PZ: periodic transverse axes (compile-time, so the removal test at the
// faces is a fixed instruction sequence).
template <int D, int ORDER, bool PY, bool PZ, bool LOCAL, class IT>
__device__ __forceinline__ void push_body(const IT& I, const PushFields& f, const float* sF, int fx0,
                                          int fy0, int fz0, const GSink<PY, PZ>& gs, const LSink<D>& ls,
                                          unsigned q, uint8_t kind, int ci, int cj, int ck, uint32_t o0,
                                          uint32_t o1, uint32_t o2, float ux, float uy, float uz, int& xlo,
                                          int& xhi) {
  // ---- gather E^n, b^n
  float ex, ey, ez, bx, by, bz;
  {
    const float t0 = off_lo(o0), t1 = off_lo(o1), t2 = off_lo(o2);
    Axis<ORDER> X, Y, Z;
    if (LOCAL) {
      constexpr int N = FWin<D>::N;
      make_axis_l<ORDER>(X, ci, t0, fx0, 1);
      if (D >= 2) make_axis_l<ORDER>(Y, cj, t1, fy0, FWin<D>::X);
      if (D >= 3) make_axis_l<ORDER>(Z, ck, t2, fz0, FWin<D>::X * FWin<D>::Y);
      ex = gather_l<D, ORDER>(sF + 0 * N, X, Y, Z, 1, 0, 0);
      ey = gather_l<D, ORDER>(sF + 1 * N, X, Y, Z, 0, 1, 0);
      ez = gather_l<D, ORDER>(sF + 2 * N, X, Y, Z, 0, 0, 1);
      bx = gather_l<D, ORDER>(sF + 3 * N, X, Y, Z, 0, 1, 1);
      by = gather_l<D, ORDER>(sF + 4 * N, X, Y, Z, 1, 0, 1);
      bz = gather_l<D, ORDER>(sF + 5 * N, X, Y, Z, 1, 1, 0);
    } else {
      make_axis<ORDER>(X, ci, t0, I.nx, 0, G, 1);
      if (D >= 2) make_axis<ORDER>(Y, cj, t1, I.ny, PY, I.Gy, I.sy);
      if (D >= 3) make_axis<ORDER>(Z, ck, t2, I.nz, PZ, I.Gz, I.sz);
      ex = gather<D, ORDER>(f.E0, X, Y, Z, 1, 0, 0);
      ey = gather<D, ORDER>(f.E1, X, Y, Z, 0, 1, 0);
      ez = gather<D, ORDER>(f.E2, X, Y, Z, 0, 0, 1);
      bx = gather<D, ORDER>(f.B0, X, Y, Z, 0, 1, 1);
      by = gather<D, ORDER>(f.B1, X, Y, Z, 1, 0, 1);
      bz = gather<D, ORDER>(f.B2, X, Y, Z, 1, 1, 0);
    }
  }
  // ---- relativistic Boris (u = gamma v / c, b = c B, h = q dt / 2 m c)
  const float h = I.kh[kind];
  const float umx = ux + h * ex, umy = uy + h * ey, umz = uz + h * ez;
  const float gm = sqrtf(1.0f + umx * umx + umy * umy + umz * umz);
  const float hg = h / gm;
  const float tx = hg * bx, ty = hg * by, tz = hg * bz;
  const float sf = 2.0f / (1.0f + tx * tx + ty * ty + tz * tz);
  const float vx = umx + (umy * tz - umz * ty);
  const float vy = umy + (umz * tx - umx * tz);
  const float vz = umz + (umx * ty - umy * tx);
  ux = umx + sf * (vy * tz - vz * ty) + h * ex;
  uy = umy + sf * (vz * tx - vx * tz) + h * ey;
  uz = umz + sf * (vx * ty - vy * tx) + h * ez;
  if (!(fabsf(ux) + fabsf(uy) + fabsf(uz) <= 3.0e38f)) atomicOr(I.health, HEALTH_NONFINITE);
  const float ig = 1.0f / sqrtf(1.0f + ux * ux + uy * uy + uz * uz);
  // ---- move: integer cell + 32-bit fraction, at most one cell per step; the
  // displacement is rounded to 2^-31 cells (|disp| < 1 fits an int32 there)
  int ni = ci, nj = cj, nk = ck;
  uint32_t n0 = o0, n1 = o1, n2 = o2;
  auto move = [&](uint32_t& o, int& c, float disp) {
    disp = fminf(fmaxf(disp, -0x1.fffffep-1f), 0x1.fffffep-1f);
    const int64_t pos = (int64_t)o + 2 * (int64_t)__float2int_rn(disp * 0x1p31f);
    c += (int)(pos >> 32);
    o = (uint32_t)pos;
  };
  move(n0, ni, I.C[0] * ux * ig);
  if (D >= 2) move(n1, nj, I.C[1] * uy * ig);
  if (D >= 3) move(n2, nk, I.C[2] * uz * ig);
  // ---- Esirkepov deposit of J^{n+1/2} (scaled: dt J / eps0, V/m)
  {
    Esk<ORDER> exk, eyk, ezk;
    esk_axis<ORDER>(exk, ci, o0, ni, n0);
    if (D >= 2) esk_axis<ORDER>(eyk, cj, o1, nj, n1);
    if (D >= 3) esk_axis<ORDER>(ezk, ck, o2, nk, n2);
    const float qx = I.kq[kind][0], qy = I.kq[kind][1], qz = I.kq[kind][2];
    if (LOCAL) deposit<D, ORDER>(ls, exk, eyk, ezk, qx, qy, qz, uy * ig, uz * ig);
    else deposit<D, ORDER>(gs, exk, eyk, ezk, qx, qy, qz, uy * ig, uz * ig);
  }
  // ---- boundaries: outflow removes, periodic wraps
  bool dead = ni < 0 || ni >= I.nx;
  if (D >= 2) {
    if (PY) nj = wrapi(nj, I.ny, 1);
    else dead = dead || nj < 0 || nj >= I.ny;
  }
  if (D >= 3) {
    if (PZ) nk = wrapi(nk, I.nz, 1);
    else dead = dead || nk < 0 || nk >= I.nz;
  }
  if (dead) {
    gp(I.pkind)[q] = DEAD;
    return;
  }
  xlo = min(xlo, ni);
  xhi = max(xhi, ni);
  gp(I.pcell)[q] = pack_cell(D, ni, nj, nk);
  gp(I.po0)[q] = n0;
  if (D >= 2) gp(I.po1)[q] = n1;
  if (D >= 3) gp(I.po2)[q] = n2;
  gp(I.pu0)[q] = ux;
  gp(I.pu1)[q] = uy;
  gp(I.pu2)[q] = uz;
}

// A charged particle's state as the push reads it (kind DEAD: no particle).
struct PState {
  unsigned q;
  uint8_t kind;
  uint32_t pc, t0, t1, t2;
  float ux, uy, uz;
};

template <int D, class IT>
__device__ __forceinline__ PState load_particle(const IT& I, int p, bool valid) {
  PState s{};
  s.q = (unsigned)p;
  s.kind = valid ? gp(I.pkind)[s.q] : DEAD;
  if (s.kind == DEAD) return s;
  s.pc = gp(I.pcell)[s.q];
  s.t0 = gp(I.po0)[s.q];
  s.t1 = D >= 2 ? gp(I.po1)[s.q] : 0u;
  s.t2 = D >= 3 ? gp(I.po2)[s.q] : 0u;
  s.ux = gp(I.pu0)[s.q];
  s.uy = gp(I.pu1)[s.q];
  s.uz = gp(I.pu2)[s.q];
  return s;
}

// One charged particle (its state loaded).  TILED: the block holds the LDS
// windows of the tile with origin (tx0, ty0, tz0); a particle that started the
// step outside that tile goes through HBM and is counted as a drifter.
template <int D, int ORDER, bool PY, bool PZ, bool TILED, class IT>
__device__ __forceinline__ void push_loaded(const IT& I, const PushFields& f, const float* sF,
                                            const GSink<PY, PZ>& gs, const LSink<D>& ls, int tx0, int ty0,
                                            int tz0, const PState& st, int& xlo, int& xhi) {
  if (st.kind == DEAD) return;
  const unsigned q = st.q;
  const uint8_t kind = st.kind;
  int ci, cj, ck;
  unpack_cell(D, st.pc, ci, cj, ck);
  const uint32_t t0 = st.t0, t1 = st.t1, t2 = st.t2;
  const float ux = st.ux, uy = st.uy, uz = st.uz;
  if (TILED) {
    bool in = ci >= tx0 && ci < tx0 + ptile_ext(D, 0);
    if (D >= 2) in = in && cj >= ty0 && cj < ty0 + ptile_ext(D, 1);
    if (D >= 3) in = in && ck >= tz0 && ck < tz0 + ptile_ext(D, 2);
    if (in) {
      push_body<D, ORDER, PY, PZ, true>(I, f, sF, tx0 - 1, ty0 - 1, tz0 - 1, gs, ls, q, kind, ci, cj, ck,
                                        t0, t1, t2, ux, uy, uz, xlo, xhi);
    } else {
      const unsigned long long m = __ballot(1);
      if ((threadIdx.x & 63) == __ffsll((long long)m) - 1) atomicAdd(I.sctl + SC_NDRIFT, __popcll(m));
      push_body<D, ORDER, PY, PZ, false>(I, f, sF, 0, 0, 0, gs, ls, q, kind, ci, cj, ck, t0, t1, t2, ux,
                                         uy, uz, xlo, xhi);
    }
  } else {
    push_body<D, ORDER, PY, PZ, false>(I, f, sF, 0, 0, 0, gs, ls, q, kind, ci, cj, ck, t0, t1, t2, ux, uy,
                                       uz, xlo, xhi);
  }
}

// One charged particle (slot p): load, then push.  In 1D and 2D the loads
// stay inside the push as one body: the split into load_particle and
// push_loaded costs the 2D push 10 % (different registers and schedule).
template <int D, int ORDER, bool PY, bool PZ, bool TILED, class IT>
__device__ __forceinline__ void push_one(const IT& I, const PushFields& f, const float* sF,
                                         const GSink<PY, PZ>& gs, const LSink<D>& ls, int tx0, int ty0,
                                         int tz0, int p, bool valid, int& xlo, int& xhi) {
  if (D == 3) {
    push_loaded<D, ORDER, PY, PZ, TILED>(I, f, sF, gs, ls, tx0, ty0, tz0, load_particle<D>(I, p, valid), xlo, xhi);
    return;
  }
  const unsigned q = (unsigned)p;
  const uint8_t kind = valid ? gp(I.pkind)[q] : DEAD;
  if (kind == DEAD) return;
  int ci, cj, ck;
  unpack_cell(D, gp(I.pcell)[q], ci, cj, ck);
  const uint32_t t0 = gp(I.po0)[q];
  const uint32_t t1 = D >= 2 ? gp(I.po1)[q] : 0u;
  const uint32_t t2 = D >= 3 ? gp(I.po2)[q] : 0u;
  const float ux = gp(I.pu0)[q], uy = gp(I.pu1)[q], uz = gp(I.pu2)[q];
  if (TILED) {
    bool in = ci >= tx0 && ci < tx0 + ptile_ext(D, 0);
    if (D >= 2) in = in && cj >= ty0 && cj < ty0 + ptile_ext(D, 1);
    if (D >= 3) in = in && ck >= tz0 && ck < tz0 + ptile_ext(D, 2);
    if (in) {
      push_body<D, ORDER, PY, PZ, true>(I, f, sF, tx0 - 1, ty0 - 1, tz0 - 1, gs, ls, q, kind, ci, cj, ck,
                                        t0, t1, t2, ux, uy, uz, xlo, xhi);
    } else {
      const unsigned long long m = __ballot(1);
      if ((threadIdx.x & 63) == __ffsll((long long)m) - 1) atomicAdd(I.sctl + SC_NDRIFT, __popcll(m));
      push_body<D, ORDER, PY, PZ, false>(I, f, sF, 0, 0, 0, gs, ls, q, kind, ci, cj, ck, t0, t1, t2, ux,
                                         uy, uz, xlo, xhi);
    }
  } else {
    push_body<D, ORDER, PY, PZ, false>(I, f, sF, 0, 0, 0, gs, ls, q, kind, ci, cj, ck, t0, t1, t2, ux, uy,
                                       uz, xlo, xhi);
  }
}

// Slot of particle i of a work item: first the sorted range [lo, hi), then the
// tile's births since the sort -- f electrons from b0 on and their f positive
// carriers from b0 + cap on (cap = the tile's birth capacity).
__device__ __forceinline__ int item_slot(int i, int lo, int n_sorted, int b0, int f, int cap) {
  if (i < n_sorted) return lo + i;
  const int j = i - n_sorted;
  return j < f ? b0 + j : b0 + cap + (j - f);
}

// Charged-particle phase.  Work items of a block (persistent grid-stride):
// first the chunks of the sorted tiles -- the block stages the tile's field
// window in LDS and clears its current window, pushes the chunk's particles
// (the tile's last chunk also its births since the sort), then adds the
// current window's nonzero nodes to HBM with one atomic each -- then the
// unsorted tail (particles placed or born beyond the tiles' layout) through
// HBM.  ONE: a single run, its parameter block passed by value.
template <int D, int ORDER, bool PY, bool PZ, bool ONE>
__global__ __launch_bounds__(push_tpb(D), D == 3 ? 4 : 1) void k_push(Group g, std::conditional_t<ONE, Inst, NoInst> one) {
  constexpr int NT = push_tpb(D);
  __shared__ unsigned long long sJ[3 * PWin<D>::N];
  __shared__ float sF[6 * FWin<D>::N];
  const Slot sl = ONE ? Slot{0, (int)blockIdx.x, g.blocks} : block_slot(g);
  auto& I = inst_of(g, sl.ii, one);
  const int nb = sl.nbk;
  const int b0 = sl.bk;
  int count = *I.pcount;
  count = count < I.capacity ? count : I.capacity;
  const int step = ONE || g.step >= 0 ? g.step : I.step_now;
  const int par = step & 1;
  int xlo = 1 << 30, xhi = -(1 << 30);   // x cells of this block's particles after the move
  const PushFields f{uniform(I.F[par][0]), uniform(I.F[par][1]), uniform(I.F[par][2]),
                     uniform(I.F[par][3]), uniform(I.F[par][4]), uniform(I.F[par][5])};
  const GSink<PY, PZ> gs{I.Jb[par][0], I.Jb[par][1], I.Jb[par][2], I.ny, I.nz, I.sy, I.sz, I.Gy, I.Gz};
  int nsorted = I.sctl[SC_NSORTED];
  nsorted = nsorted < count ? nsorted : count;
  const int nchunks = I.sctl[SC_NCHUNKS];
  const int64_t ncell = (int64_t)I.Px * I.Py * I.Pz;
  // one work item: a chunk of a sorted tile
  auto work = [&](int v) {
    const int4 ch = I.chunks[v];
    const int t = ch.x;
    const int n_sorted = ch.z - ch.y;
    int nbirth = 0, bcap = 0;
    if (ch.w >= 0) {
      bcap = I.tslack[t];
      const int fe = I.tfill[t];
      nbirth = fe < bcap ? fe : bcap;
    }
    const int ntot = n_sorted + 2 * nbirth;
    if (ntot == 0) return;
    if (ntot <= sparse_chunk(D)) {
      // a sparse piece (one pass of the block): HBM atomics cost less than
      // staging and flushing the windows
      const int i = threadIdx.x;
      const int p = i < ntot ? item_slot(i, ch.y, n_sorted, ch.w, nbirth, bcap) : 0;
      push_one<D, ORDER, PY, PZ, false>(I, f, sF, gs, LSink<D>{sJ, 0, 0, 0, 0.0}, 0, 0, 0, p, i < ntot,
                                        xlo, xhi);
      return;
    }
    const int tx0 = (t % I.ntile[0]) * ptile_ext(D, 0);
    const int ty0 = D >= 2 ? ((t / I.ntile[0]) % I.ntile[1]) * ptile_ext(D, 1) : 0;
    const int tz0 = D >= 3 ? (t / (I.ntile[0] * I.ntile[1])) * ptile_ext(D, 2) : 0;
    const LSink<D> ls{sJ, tx0 - PT_LO, D >= 2 ? ty0 - PT_LO : 0, D >= 3 ? tz0 - PT_LO : 0,
                      (double)I.jscale};
    // 3D: the first pass's particles load while the windows are cleared and
    // staged (in 2D the registers this holds cost more than the overlap gains)
    PState first{};
    if (D == 3)
      first = load_particle<D>(I, (int)threadIdx.x < ntot ? item_slot(threadIdx.x, ch.y, n_sorted, ch.w, nbirth, bcap) : 0,
                               (int)threadIdx.x < ntot);
    for (int e = threadIdx.x; e < 3 * PWin<D>::N; e += NT) sJ[e] = 0ull;
    // field window: nodes tile - 1 .. tile + T + 1 (periodic axes wrapped;
    // nodes outside the padded arrays, never read, are zero).  Threads walk
    // the window row by row: a row of X nodes per (b, c).
    constexpr int FX = FWin<D>::X, FY = FWin<D>::Y;
    for (int e = threadIdx.x; e < FWin<D>::N; e += NT) {
      const int a = e % FX;
      const int r = e / FX;
      const int b = D >= 2 ? r % FY : 0;
      const int c = D >= 3 ? r / FY : 0;
      const int px = tx0 - 1 + a + G;
      bool ok = px < I.Px;
      int off = px;
      if (D >= 2) {
        int j = ty0 - 1 + b;
        if (PY) j = j < 0 ? j + I.ny : (j >= I.ny ? j - I.ny : j);
        ok = ok && j + I.Gy < I.Py;
        off += I.sy * (j + I.Gy);
      }
      if (D >= 3) {
        int k = tz0 - 1 + c;
        if (PZ) k = k < 0 ? k + I.nz : (k >= I.nz ? k - I.nz : k);
        ok = ok && k + I.Gz < I.Pz;
        off += I.sz * (k + I.Gz);
      }
      const unsigned o = (unsigned)off;
      sF[0 * FWin<D>::N + e] = ok ? gp(f.E0)[o] : 0.0f;
      sF[1 * FWin<D>::N + e] = ok ? gp(f.E1)[o] : 0.0f;
      sF[2 * FWin<D>::N + e] = ok ? gp(f.E2)[o] : 0.0f;
      sF[3 * FWin<D>::N + e] = ok ? gp(f.B0)[o] : 0.0f;
      sF[4 * FWin<D>::N + e] = ok ? gp(f.B1)[o] : 0.0f;
      sF[5 * FWin<D>::N + e] = ok ? gp(f.B2)[o] : 0.0f;
    }
    __syncthreads();
    if (D == 3) push_loaded<D, ORDER, PY, PZ, true>(I, f, sF, gs, ls, tx0, ty0, tz0, first, xlo, xhi);
    for (int i0 = D == 3 ? NT : 0; i0 < ntot; i0 += NT) {
      const int i = i0 + threadIdx.x;
      const int p = i < ntot ? item_slot(i, ch.y, n_sorted, ch.w, nbirth, bcap) : 0;
      push_one<D, ORDER, PY, PZ, true>(I, f, sF, gs, ls, tx0, ty0, tz0, p, i < ntot, xlo, xhi);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 3 * PWin<D>::N; e += NT) {
      const unsigned long long raw = sJ[e];
      if (raw == 0ull) continue;
      const float v = (float)(double)(long long)raw * I.jscale_inv;
      const int comp = e / PWin<D>::N;
      const int r = e - comp * PWin<D>::N;
      const int a = r % PWin<D>::X;
      const int b = (r / PWin<D>::X) % PWin<D>::Y;
      const int c = r / (PWin<D>::X * PWin<D>::Y);
      const int o = gs.x(ls.x0 + a) + (D >= 2 ? gs.y(ls.y0 + b) : 0) + (D >= 3 ? gs.z(ls.z0 + c) : 0);
      if (o >= 0 && o < ncell) gs.put(comp, o, v, 1.0f);
    }
  };
  // Work queues: the chunk list in 8 contiguous ranges, one per XCD (a block
  // runs on XCD blockIdx.x mod 8), so neighbouring tiles share that XCD's L2.
  // A block takes the next chunk of its own range (one atomic, issued while
  // it works on the current chunk); when the range is used up it reads all
  // eight counters at once and moves to a range with chunks left.  The grid
  // is the number of blocks resident at once: work goes to whichever block is
  // free, so chunks of very different sizes leave no block idle (blocks past
  // the chunk count take no part).  The last block out of those taking part
  // clears the counters for the next launch.
  __shared__ int s_next;
  __shared__ int s_left[8];
  auto range = [&](int x, int& lo, int& hi) {
    lo = (int)((int64_t)nchunks * x / 8);
    hi = (int)((int64_t)nchunks * (x + 1) / 8);
  };
  if (b0 < nchunks) {
    int xq = (int)(blockIdx.x & 7u);
    while (true) {
      int lo, hi;
      range(xq, lo, hi);
      int* const ctr = I.pq + 64 * xq;
      if (threadIdx.x == 0) s_next = lo < hi ? lo + atomicAdd(ctr, 1) : hi;
      __syncthreads();
      int v = s_next;
      while (v < hi) {
        int nxt = 0;
        if (threadIdx.x == 0) nxt = lo + atomicAdd(ctr, 1);   // the next item, in flight meanwhile
        work(v);
        __syncthreads();   // the windows are free again, and s_next has been read
        if (threadIdx.x == 0) s_next = nxt;
        __syncthreads();
        v = s_next;
      }
      if (threadIdx.x < 8) {
        int l, h;
        range((int)threadIdx.x, l, h);
        s_left[threadIdx.x] = (h - l) - __hip_atomic_load(I.pq + 64 * threadIdx.x, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
      }
      __syncthreads();
      int pick = -1;
      for (int k = 1; k <= 8 && pick < 0; ++k)
        if (s_left[(xq + k) & 7] > 0) pick = (xq + k) & 7;
      __syncthreads();
      if (pick < 0) break;
      xq = pick;
    }
    // the last of the min(nb, nchunks) taking part clears the counters
    if (threadIdx.x == 0) {
      __threadfence();
      if (atomicAdd(I.pq + 64 * 8, 1) == min(nb, nchunks) - 1) {
        for (int x = 0; x <= 8; ++x) __hip_atomic_store(I.pq + 64 * x, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
      }
    }
  }
  const LSink<D> none{sJ, 0, 0, 0, 0.0};
  for (int p0 = nsorted + b0 * NT; p0 < count; p0 += nb * NT) {
    const int p = p0 + threadIdx.x;
    push_one<D, ORDER, PY, PZ, false>(I, f, sF, gs, none, 0, 0, 0, p, p < count, xlo, xhi);
  }
  // charged region of the next step: this step's region plus where this
  // block's particles went (an atomic only where a block extends it)
  __shared__ int sxr[2][NT / 64];
  for (int o = 32; o > 0; o >>= 1) {
    xlo = min(xlo, __shfl_xor(xlo, o));
    xhi = max(xhi, __shfl_xor(xhi, o));
  }
  if ((threadIdx.x & 63) == 0) {
    sxr[0][threadIdx.x >> 6] = xlo;
    sxr[1][threadIdx.x >> 6] = xhi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < NT / 64; ++w) {
      xlo = min(xlo, sxr[0][w]);
      xhi = max(xhi, sxr[1][w]);
    }
    const int* cur = I.xext + 2 * (step % 3);
    int* nxt = I.xext + 2 * ((step + 1) % 3);
    const int clo = cur[0], chi = cur[1];
    if (b0 == 0) {
      atomicMin(nxt, min(clo, xlo));
      atomicMax(nxt + 1, max(chi, xhi));
    } else {
      if (xlo < clo) atomicMin(nxt, xlo);
      if (xhi > chi) atomicMax(nxt + 1, xhi);
    }
  }
}

// ------------------------------------------------------------ tile sort
// Counting sort of the charged particles by tile: count (wave-aggregated
// atomics), scan (one block per instance: the tiles' ranges, each followed by
// its birth capacity, and the chunk list), fill (every slot of the new layout
// starts empty), scatter into the spare arrays (dead slots dropped), copy back.
// A tile's births until the next sort go into its capacity: electrons and
// positive carriers in two halves of one alive-neutral bound each (neutrals do
// not move and ionize once, so the bound is never exceeded).  The first kernel
// decides, identically in every block, whether a sort is due; the others
// follow its decision.
template <int D, class IT>
__device__ __forceinline__ int tile_of(const IT& I, uint32_t pc) {
  int i, j, k;
  unpack_cell(D, pc, i, j, k);
  constexpr int TX = ptile_ext(D, 0), TY = ptile_ext(D, 1), TZ = ptile_ext(D, 2);
  int t = i / TX;
  if (D >= 2) t += I.ntile[0] * (j / TY);
  if (D >= 3) t += I.ntile[0] * I.ntile[1] * (k / TZ);
  return (unsigned)t < (unsigned)I.ntiles ? t : -1;   // -1 only for a corrupt cell
}

// Adds k to arr[t] for every lane with t >= 0, one atomic per distinct t of the
// wave; returns the lane's offset (distinct multiples of k per lane and t).
__device__ __forceinline__ int wave_rank_add(int* arr, int t, int k = 1) {
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  unsigned long long pending = __ballot(t >= 0);
  int rank = 0;
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const int tl = __shfl(t, leader);
    const unsigned long long m = __ballot(t == tl);
    int base = 0;
    if (lane == leader) base = atomicAdd(arr + tl, k * __popcll(m));
    base = __shfl(base, leader);
    if (t == tl) rank = base + k * __popcll(m & below);
    pending &= ~m;
  }
  return rank;
}

template <int D>
__global__ __launch_bounds__(TPB) void k_sort_count(Group g) {
  const int ii = find_inst(g);
  auto& I = inst_of(g, ii, NoInst{});
  const int nb = g.off[ii + 1] - g.off[ii];
  const int b0 = blockIdx.x - g.off[ii];
  int count = *I.pcount;
  count = count < I.capacity ? count : I.capacity;
  const int loose = count - I.sctl[SC_NSORTED];
  const int drift = I.sctl[SC_NDRIFT];
  // forced (a new layout is wanted), particles beyond the layout above 1/32 of
  // the slots, or drifter-steps (per step, a particle deposited outside its
  // tile) above 1/16
  const int lo = count >> 5, dr = count >> 4;
  const int go = I.sctl[SC_FORCE] || loose > (lo > 256 ? lo : 256) || drift > (dr > 256 ? dr : 256);
  if (b0 == 0 && threadIdx.x == 0) I.sctl[SC_GO] = go;
  if (!go) return;
  const int lane = threadIdx.x & 63;
  for (int p0 = b0 * TPB + (threadIdx.x - lane); p0 < count; p0 += nb * TPB) {
    const int p = p0 + lane;
    const int t = p < count && I.pkind[p] != DEAD ? tile_of<D>(I, I.pcell[p]) : -1;
    (void)wave_rank_add(I.tcnt, t);
  }
}

constexpr int SCAN_TPB = 1024;

template <int D>
__global__ __launch_bounds__(SCAN_TPB) void k_sort_scan(Group g) {
  constexpr int TPB = SCAN_TPB;
  __shared__ long long sp[TPB], sc[TPB];
  __shared__ int sfit;
  const int ii = find_inst(g);
  auto& I = inst_of(g, ii, NoInst{});
  if (!I.sctl[SC_GO]) return;
  const int nt = I.ntiles;
  const int per = (nt + TPB - 1) / TPB;
  const int t0 = threadIdx.x * per;
  const int t1 = t0 + per < nt ? t0 + per : nt;
  // births since the sort used up alive neutrals: the bound of each tile drops
  // by the births its capacity took (births beyond it went to the tail and are
  // not counted, which keeps the bound an upper bound)
  long long np = 0, nc = 0, ns = 0;
  for (int t = t0; t < t1; ++t) {
    const int cap = I.tslack[t];
    const int fe = I.tfill[t];
    const int alive = I.talive[t] - (fe < cap ? fe : cap);
    I.talive[t] = alive;
    const int n = I.tcnt[t];
    np += n;
    ns += 2 * (long long)alive;
  }
  sp[threadIdx.x] = np;
  sc[threadIdx.x] = ns;
  __syncthreads();
  for (int w = 1; w < TPB; w <<= 1) {   // inclusive scans
    const long long a = threadIdx.x >= w ? sp[threadIdx.x - w] : 0;
    const long long b = threadIdx.x >= w ? sc[threadIdx.x - w] : 0;
    __syncthreads();
    sp[threadIdx.x] += a;
    sc[threadIdx.x] += b;
    __syncthreads();
  }
  // birth capacity only when the whole layout fits the slots
  if (threadIdx.x == 0) sfit = sp[TPB - 1] + sc[TPB - 1] <= (long long)I.capacity;
  __syncthreads();
  const bool fit = sfit;
  long long pp = (sp[threadIdx.x] - np) + (fit ? sc[threadIdx.x] - ns : 0);
  for (int t = t0; t < t1; ++t) {
    const int n = I.tcnt[t];
    const int cap = fit ? I.talive[t] : 0;
    nc += (n + SORT_CHUNK - 1) / SORT_CHUNK + (n == 0 && cap > 0);
  }
  __syncthreads();
  sc[threadIdx.x] = nc;
  __syncthreads();
  for (int w = 1; w < TPB; w <<= 1) {
    const long long b = threadIdx.x >= w ? sc[threadIdx.x - w] : 0;
    __syncthreads();
    sc[threadIdx.x] += b;
    __syncthreads();
  }
  long long pc = sc[threadIdx.x] - nc;
  const long long tchunks = sc[TPB - 1];
  for (int t = t0; t < t1; ++t) {
    const int n = I.tcnt[t];
    const int cap = fit ? I.talive[t] : 0;
    const long long ts = pp;
    const int bl = (int)(ts + n);   // first birth slot
    // slot order inside the tile: the particles the scatter ranks r = 0, 1, ...
    // (arriving roughly cell by cell) go to slots (r P) mod n, P coprime with n
    // and near n / 64, so the 64 lanes of a wave hold particles from all over
    // the tile: few lanes share a cell, and few LDS atomics of one
    // instruction hit the same node (same-node lanes serialise)
    int P = 1;
    if (n >= 128) {
      P = (n >> 6) | 1;
      for (;;) {
        int a = P, b = n;
        while (b) {
          const int r = a % b;
          a = b;
          b = r;
        }
        if (a == 1) break;
        P += 2;
      }
    }
    I.tperm[t] = P;
    I.tcnt[t] = 0;              // the scatter's rank counter
    I.tstart[t] = (int)ts;
    I.tbirth[t] = bl;
    I.tslack[t] = cap;
    I.tfill[t] = 0;
    pp += n + 2 * (long long)cap;
    if (n == 0) {
      if (cap > 0) I.chunks[pc++] = make_int4(t, (int)ts, (int)ts, bl);
      continue;
    }
    for (long long q = 0; q * SORT_CHUNK < n; ++q) {
      const long long e = (q + 1) * SORT_CHUNK;
      const bool last = e >= n;
      I.chunks[pc++] = make_int4(t, (int)(ts + q * SORT_CHUNK), (int)(ts + (last ? n : e)),
                                 last && cap > 0 ? bl : -1);
    }
  }
  __syncthreads();
  if (threadIdx.x == TPB - 1) {
    // the layout's end: tiles and their birth room (the live particles alone
    // always fit the slots)
    I.sctl[SC_NSORTED] = (int)(pp < (long long)I.capacity ? pp : (long long)I.capacity);
    I.sctl[SC_NCHUNKS] = (int)tchunks;
    I.sctl[SC_FORCE] = 0;
  }
}

// Every slot of the new layout starts empty (its kind DEAD in the spare array).
// The layout never exceeds the slots (the live particles fit, and the birth
// room is only laid out when it fits too); the bound is kept here regardless.
template <int D>
__global__ __launch_bounds__(TPB) void k_sort_fill(Group g) {
  const int ii = find_inst(g);
  auto& I = inst_of(g, ii, NoInst{});
  if (!I.sctl[SC_GO]) return;
  const int nb = g.off[ii + 1] - g.off[ii];
  const int b0 = blockIdx.x - g.off[ii];
  const int n = min(I.sctl[SC_NSORTED], I.capacity);
  for (int p = b0 * TPB + threadIdx.x; p < n; p += nb * TPB) I.skind[p] = DEAD;
}

template <int D>
__global__ __launch_bounds__(TPB) void k_sort_scatter(Group g) {
  const int ii = find_inst(g);
  auto& I = inst_of(g, ii, NoInst{});
  if (!I.sctl[SC_GO]) return;
  const int nb = g.off[ii + 1] - g.off[ii];
  const int b0 = blockIdx.x - g.off[ii];
  int count = *I.pcount;
  count = count < I.capacity ? count : I.capacity;
  const int lane = threadIdx.x & 63;
  for (int p0 = b0 * TPB + (threadIdx.x - lane); p0 < count; p0 += nb * TPB) {
    const int p = p0 + lane;
    int t = -1;
    uint32_t pc = 0;
    uint8_t kd = DEAD;
    if (p < count) {
      kd = I.pkind[p];
      pc = I.pcell[p];
      if (kd != DEAD) t = tile_of<D>(I, pc);
    }
    const int r = wave_rank_add(I.tcnt, t);
    if (t < 0) continue;
    const int ts = I.tstart[t];
    const unsigned n = (unsigned)(I.tbirth[t] - ts);
    const int d = ts + (int)(((unsigned long long)(unsigned)r * (unsigned)I.tperm[t]) % n);
    if ((unsigned)d >= (unsigned)I.capacity) continue;
    I.scell[d] = pc;
    I.skind[d] = kd;
    I.so0[d] = I.po0[p];
    if (D >= 2) I.so1[d] = I.po1[p];
    if (D >= 3) I.so2[d] = I.po2[p];
    I.su0[d] = I.pu0[p];
    I.su1[d] = I.pu1[p];
    I.su2[d] = I.pu2[p];
    I.spid[d] = I.pid[p];
  }
}

// The new layout back into the particle arrays (coalesced copies); the slot
// counter becomes the layout's end, and the per-tile counters (the scatter's
// ranks) start the next sort at zero.
template <int D>
__global__ __launch_bounds__(TPB) void k_sort_copy(Group g) {
  const int ii = find_inst(g);
  auto& I = inst_of(g, ii, NoInst{});
  if (!I.sctl[SC_GO]) return;
  const int nb = g.off[ii + 1] - g.off[ii];
  const int b0 = blockIdx.x - g.off[ii];
  const int n = min(I.sctl[SC_NSORTED], I.capacity);
  for (int t = b0 * TPB + threadIdx.x; t < I.ntiles; t += nb * TPB) I.tcnt[t] = 0;
  for (int p = b0 * TPB + threadIdx.x; p < n; p += nb * TPB) {
    I.pcell[p] = I.scell[p];
    I.pkind[p] = I.skind[p];
    I.po0[p] = I.so0[p];
    if (D >= 2) I.po1[p] = I.so1[p];
    if (D >= 3) I.po2[p] = I.so2[p];
    I.pu0[p] = I.su0[p];
    I.pu1[p] = I.su1[p];
    I.pu2[p] = I.su2[p];
    I.pid[p] = I.spid[p];
  }
  if (b0 == 0 && threadIdx.x == 0) {
    *I.pcount = n;
    I.sctl[SC_NDRIFT] = 0;
    I.sctl[SC_NSORTS] += 1;
  }
}

// ------------------------------------------------------------ field solve
// First-order outflow (Mur) for a face point q with inward neighbour r:
// E_q^{n+1} = E_r^n + k (E_r^{n+1} - E_q^n), applied to the field minus the
// incident wave on the injection face.
struct MurInc {
  float q0, q1, r0, r1;   // incident field at q and r, levels n and n+1
};

__device__ __forceinline__ float mur(float qold, float rold, float rnew, float k) {
  return rold + k * (rnew - qold);
}
__device__ __forceinline__ float mur_inc(float qold, float rold, float rnew, float k, const MurInc& m) {
  return m.q1 + (rold - m.r0) + k * ((rnew - m.r1) - (qold - m.q0));
}

// Tile shapes of the field kernel (owned positions per block), per dimension.
struct TileShape {
  int x, y, z;
};
// Shapes 3 to 6 (2D, 3D) and 5, 6 (1D) make the staged row (x extent plus
// the 2 + 2 halo) a power of two, so a thread's staged index splits into
// coordinates by shifts.
__host__ __device__ constexpr TileShape tile_shape(int D, int v) {
  return D == 1 ? (v == 1 ? TileShape{128, 1, 1} : v == 2 ? TileShape{512, 1, 1} : v == 5 ? TileShape{252, 1, 1}
                   : v == 6 ? TileShape{508, 1, 1} : TileShape{256, 1, 1})
       : D == 2 ? (v == 1 ? TileShape{32, 8, 1} : v == 2 ? TileShape{64, 4, 1} : v == 3 ? TileShape{124, 4, 1}
                   : v == 4 ? TileShape{60, 4, 1} : v == 5 ? TileShape{60, 8, 1} : v == 6 ? TileShape{60, 12, 1}
                   : TileShape{64, 8, 1})
                : (v == 1 ? TileShape{12, 4, 8} : v == 2 ? TileShape{16, 4, 4} : v == 3 ? TileShape{28, 4, 4}
                   : v == 4 ? TileShape{12, 12, 4} : v == 5 ? TileShape{12, 4, 4} : v == 6 ? TileShape{12, 8, 4}
                   : v == 7 ? TileShape{60, 8, 1} : TileShape{16, 8, 4});
}
// Variant 7 (3D with periodic y and z only) is the z-marching update: x-y
// tiles of 60 x 8 positions over the box, z in segments (as many as fill the
// GPU's resident blocks).
constexpr int kTileVariants = 8;
constexpr int kMarchVariant = 7;

__device__ __forceinline__ int wrap_any(int j, int n) {
  j %= n;
  return j < 0 ? j + n : j;
}

// decode a padded linear index into logical (i, j, k)
template <int D, class IT>
__device__ __forceinline__ void decode(const IT& I, int64_t p, int& i, int& j, int& k) {
  const int ai = (int)(p % I.Px);
  const int64_t r = p / I.Px;
  const int aj = D >= 2 ? (int)(r % I.Py) : 0;
  const int ak = D >= 3 ? (int)(r / I.Py) : 0;
  i = ai - G;
  j = aj - I.Gy;
  k = ak - I.Gz;
}

// validity of a staggered position along one axis (v logical, n cells)
__device__ __forceinline__ bool v_b(int v, int n, bool half, bool per) {
  return per || (half ? (v >= 0 && v < n) : (v >= 0 && v <= n));
}
__device__ __forceinline__ bool v_in(int v, int n, bool half, bool per) {   // E interior
  return per || (half ? (v >= 0 && v < n) : (v >= 1 && v <= n - 1));
}
__device__ __forceinline__ bool v_dom(int v, int n, bool half, bool per) {  // inside the box
  return per ? (v >= 0 && v < n) : (half ? (v >= 0 && v < n) : (v >= 0 && v <= n));
}

// Lorentz oscillator at one E position: the polarisation current of the
// step from E^n and Q^n (set n & 1), returned for the E update; the block that
// owns the position stores K^{n+1/2} and Q^{n+1} = Q^n + K^{n+1/2} in set
// (n + 1) & 1.  L = (a, c, c deps).
struct LorPtrs {
  const gmem<float>* Kc;
  const gmem<float>* Qc;
  gmem<float>* Kn;
  gmem<float>* Qn;
};
// (a macro, not a function: the kernels' parameter block stays in the
// kernel-argument segment instead of being copied to private memory)
#define LOR_PTRS(I, par, c)                                                                       \
  LorPtrs { gp(uniform((I).Kp[par][c])), gp(uniform((I).Q[par][c])), gp(uniform((I).Kp[(par) ^ 1][c])), \
            gp(uniform((I).Q[(par) ^ 1][c])) }
__device__ __forceinline__ float lor_step(const LorPtrs& p, unsigned gi, float4 L, float e_old, bool own) {
  const float ko = at(p.Kc, gi), qo = at(p.Qc, gi);
  const float kn = fmaf(L.x, ko, fmaf(L.z, e_old, -L.y * qo));
  if (own) {
    at(p.Kn, gi) = kn;
    at(p.Qn, gi) = qo + kn;
  }
  return kn;
}

// E^{n+1} at a Kerr position: the displacement e / ie + chi3 e^3 advances by
// src (curl and currents); X + g X^3 = R, g = ie chi3, by Newton from the
// linear update (three steps: g X^2 is small, the start within g e^2 of it)
__device__ __forceinline__ float kerr_update(float e, float ie, float src, float chi3) {
  const float g = ie * chi3;
  const float lin = e + ie * src;
  const float R = lin + g * e * e * e;
  float X = lin;
#pragma unroll
  for (int it = 0; it < 3; ++it) X -= (X + g * X * X * X - R) / (1.0f + 3.0f * g * X * X);
  return X;
}

template <int D, int V>
struct TileT {
  static constexpr int X = tile_shape(D, V).x, Y = tile_shape(D, V).y, Z = tile_shape(D, V).z;
};

// Per-axis facts of a local tile coordinate, as bits.
enum : unsigned {
  AX_BN = 1u,     // b valid, node-staggered
  AX_BH = 2u,     // b valid, half-staggered
  AX_IN = 4u,     // E interior, node
  AX_IH = 8u,     // E interior, half
  AX_DN = 16u,    // inside the box, node
  AX_DH = 32u,    // inside the box, half
  AX_ARR = 64u,   // has a position in the padded array
  AX_F0 = 128u,   // on the min face (node index 0)
  AX_F1 = 256u    // on the max face (node index n)
};

__device__ __forceinline__ unsigned axis_bits(int v, int n, bool per, bool inarr) {
  unsigned b = inarr ? AX_ARR : 0u;
  if (per) return b | AX_BN | AX_BH | AX_IN | AX_IH | ((v >= 0 && v < n) ? (AX_DN | AX_DH) : 0u);
  if (v >= 0 && v <= n) b |= AX_BN | AX_DN;
  if (v >= 0 && v < n) b |= AX_BH | AX_IH | AX_DH;
  if (v >= 1 && v <= n - 1) b |= AX_IN;
  if (v == 0) b |= AX_F0;
  if (v == n) b |= AX_F1;
  return b;
}

// One block = one tile of owned positions plus a halo of 2 on each side of
// every present axis, all six field components staged in LDS.  Row and plane
// offsets (periodic axes wrapped) and per-axis validity bits are tabulated
// once per block.  ONE: a single run whose parameter block, step index and
// front and charged-range addresses come in the launch, so that the first
// loads of a block are one round trip instead of a chain of dependent ones.
template <int D, int V, int LOR, bool ONE>
__global__ __launch_bounds__(TPB) void k_fields(Group g, std::conditional_t<ONE, Inst, NoInst> one) {
  using T = TileT<D, V>;
  constexpr int H = 2;
  constexpr int RX = T::X + 2 * H;
  constexpr int RY = D >= 2 ? T::Y + 2 * H : 1;
  constexpr int RZ = D >= 3 ? T::Z + 2 * H : 1;
  constexpr int NR = RX * RY * RZ;
  constexpr int LY = RX, LZ = RX * RY;   // LDS strides
  __shared__ float sE[3][NR];
  __shared__ float sB[3][NR];
  __shared__ unsigned sbx[RX], sby[RY], sbz[RZ];
  __shared__ int soy[RY], soz[RZ];
  __shared__ float sieh[RX], sien[RX];
  __shared__ int blk_hot;
  constexpr int KMAX = (NR + TPB - 1) / TPB;   // staged points per thread
  const Slot sl = ONE ? Slot{0, (int)blockIdx.x, g.blocks} : block_slot(g);
  auto& I = inst_of(g, sl.ii, one);
  // step parity in a scalar register, so the field pointers load as scalars
  const int step = ONE || g.step >= 0 ? g.step : I.step_now;
  const int par = step & 1;
  // the field front (the last x column of a tile that has stored a nonzero E
  // or b) and the charged x range, first used after the axis tables.  Relaxed
  // atomic loads (plain loads in the instruction stream) are issued here and
  // not moved down to their first use; another tile raising the front during
  // this launch only makes the test below more conservative.
  int* const frontp = ONE ? g.front : I.front;
  gmem<int>* const xe = gp(const_cast<int*>(ONE ? g.xext : I.xext) + 2 * (step % 3));
  const int front = __hip_atomic_load(gp(frontp), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  const int xlo = __hip_atomic_load(xe, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  const int xhi = __hip_atomic_load(xe + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  const gmem<float>* __restrict__ Ec0 = gp(uniform(I.F[par][0]));
  const gmem<float>* __restrict__ Ec1 = gp(uniform(I.F[par][1]));
  const gmem<float>* __restrict__ Ec2 = gp(uniform(I.F[par][2]));
  const gmem<float>* __restrict__ Bc0 = gp(uniform(I.F[par][3]));
  const gmem<float>* __restrict__ Bc1 = gp(uniform(I.F[par][4]));
  const gmem<float>* __restrict__ Bc2 = gp(uniform(I.F[par][5]));
  gmem<float>* __restrict__ En0 = gp(uniform(I.F[par ^ 1][0]));
  gmem<float>* __restrict__ En1 = gp(uniform(I.F[par ^ 1][1]));
  gmem<float>* __restrict__ En2 = gp(uniform(I.F[par ^ 1][2]));
  gmem<float>* __restrict__ Bn0 = gp(uniform(I.F[par ^ 1][3]));
  gmem<float>* __restrict__ Bn1 = gp(uniform(I.F[par ^ 1][4]));
  gmem<float>* __restrict__ Bn2 = gp(uniform(I.F[par ^ 1][5]));
  const gmem<float>* __restrict__ J0 = gp(uniform(I.Jb[par][0]));
  const gmem<float>* __restrict__ J1 = gp(uniform(I.Jb[par][1]));
  const gmem<float>* __restrict__ J2 = gp(uniform(I.Jb[par][2]));
  gmem<float>* __restrict__ Jn0 = gp(uniform(I.Jb[par ^ 1][0]));
  gmem<float>* __restrict__ Jn1 = gp(uniform(I.Jb[par ^ 1][1]));
  gmem<float>* __restrict__ Jn2 = gp(uniform(I.Jb[par ^ 1][2]));
  const gmem<float>* __restrict__ ieh = gp(I.ie_half);
  const gmem<float>* __restrict__ ien = gp(I.ie_node);
  const float hx = I.halfC[0], hy = I.halfC[1], hz = I.halfC[2];
  const float Cx = I.C[0], Cy = I.C[1], Cz = I.C[2];
  const int Px = I.Px, Py = I.Py, Pz = I.Pz;
  const int ntx = (Px + T::X - 1) / T::X;
  const int nty = D >= 2 ? (Py + T::Y - 1) / T::Y : 1;
  const int nbk = sl.nbk, bk = sl.bk;
  const int nx = I.nx, ny = I.ny, nz = I.nz;
  const bool py = I.per_y, pz = I.per_z;
  const int sy = I.sy, sz = I.sz;
  const int Gy = I.Gy, Gz = I.Gz;
  auto split = [&](int l, int& qx, int& qy, int& qz) {
    qx = l % RX;
    qy = D >= 2 ? (l / RX) % RY : 0;
    qz = D >= 3 ? l / (RX * RY) : 0;
  };
  // one block per tile; each XCD walks a contiguous range of tiles
  const int tb = xcd_remap(bk, nbk);
  const int tx = tb % ntx, rest = tb / ntx;
  const int a0x = tx * T::X;
  const int a0y = D >= 2 ? (rest % nty) * T::Y : 0;
  const int a0z = D >= 3 ? (rest / nty) * T::Z : 0;
  const int i0 = a0x - G, j0 = a0y - Gy, k0 = a0z - Gz;   // logical tile origin
  // far tiles: x columns farther than XNEAR_MARGIN cells from every cell that
  // held a charged particle so far and from the amplitude window have carried
  // no current, ever, so their update neither reads nor clears it
  bool cur = true;
  if (g.part >= 1) {
    int lo = xlo, hi = xhi;
    if (I.wx1 > I.wx0) {
      lo = min(lo, I.wx0 - G);
      hi = max(hi, I.wx1 - 1 - G);
    }
    const int alo = lo - XNEAR_MARGIN + G, ahi = hi + XNEAR_MARGIN + G;
    cur = lo <= hi && tx * T::X <= ahi && tx * T::X + T::X - 1 >= alo;
  }
  // a far tile whose staged x range lies beyond the front has zero inputs
  // (the update moves the front by at most two cells per step): its outputs
  // are zero and already stored, as it was skipped or wrote zeros at every
  // earlier step, so it is not updated (decided before the axis tables)
  if (g.part == 1 && !cur && a0x - H > front) return;
  if (threadIdx.x == 0) blk_hot = 0;
  // Lorentz media inside the staged x range
  const bool lorT = LOR && I.lx0 < I.lx1 && a0x - H < I.lx1 && a0x + T::X + H > I.lx0;
  // ---- per-axis tables; an interior tile (every staged position valid for
  // both updates and on no face, every owned position inside the box) runs
  // the phases below without any per-position test
  constexpr unsigned REQ = AX_ARR | AX_BN | AX_BH | AX_IN | AX_IH;
  auto interior = [](unsigned b, int q, int t) {
    return (b & REQ) == REQ && !(b & (AX_F0 | AX_F1)) &&
           (q < H || q >= t + H || (b & (AX_DN | AX_DH)) == (AX_DN | AX_DH));
  };
  bool ok = true;
  for (int q = threadIdx.x; q < RX; q += TPB) {
    const int i = i0 + q - H;
    sbx[q] = axis_bits(i, nx, false, i + G >= 0 && i + G < Px);
    ok = ok && interior(sbx[q], q, T::X);
  }
  for (int q = threadIdx.x; q < RY; q += TPB) {
    if (D >= 2) {
      const int j = j0 + q - H;
      const int jw = py ? wrap_any(j, ny) : j;
      const bool in = jw + G >= 0 && jw + G < Py;
      sby[q] = axis_bits(j, ny, py, in);
      soy[q] = in ? sy * (jw + G) : 0;
      ok = ok && interior(sby[q], q, T::Y);
    } else {
      sby[q] = AX_BN | AX_BH | AX_IN | AX_IH | AX_DN | AX_DH | AX_ARR;
      soy[q] = 0;
    }
  }
  for (int q = threadIdx.x; q < RZ; q += TPB) {
    if (D >= 3) {
      const int k = k0 + q - H;
      const int kw = pz ? wrap_any(k, nz) : k;
      const bool in = kw + G >= 0 && kw + G < Pz;
      sbz[q] = axis_bits(k, nz, pz, in);
      soz[q] = in ? sz * (kw + G) : 0;
      ok = ok && interior(sbz[q], q, T::Z);
    } else {
      sbz[q] = AX_BN | AX_BH | AX_IN | AX_IH | AX_DN | AX_DH | AX_ARR;
      soz[q] = 0;
    }
  }
  const bool inner = __syncthreads_and(ok);
  // ---- A: stage E^n and b^n; the current of the points this thread updates
  // in phase C is loaded now too (registers), so HBM latency is met once
  float jr[KMAX][3];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    const int l = threadIdx.x + k * TPB;
    if (l >= NR) continue;
    int qx, qy, qz;
    split(l, qx, qy, qz);
    const bool in = inner || (sbx[qx] & sby[qy] & sbz[qz] & AX_ARR);
    // 32-bit element offsets from uniform bases (every grid has < 2^31 points)
    const unsigned gi = (unsigned)(a0x + qx - H + soy[qy] + soz[qz]);
    sE[0][l] = in ? at(Ec0, gi) : 0.0f;
    sE[1][l] = in ? at(Ec1, gi) : 0.0f;
    sE[2][l] = in ? at(Ec2, gi) : 0.0f;
    sB[0][l] = in ? at(Bc0, gi) : 0.0f;
    sB[1][l] = in ? at(Bc1, gi) : 0.0f;
    sB[2][l] = in ? at(Bc2, gi) : 0.0f;
    const bool cpt = cur && in && qx >= H - 1 && qx <= T::X + H && (D < 2 || (qy >= H - 1 && qy <= T::Y + H)) &&
                     (D < 3 || (qz >= H - 1 && qz <= T::Z + H));
    jr[k][0] = cpt ? at(J0, gi) : 0.0f;
    jr[k][1] = cpt ? at(J1, gi) : 0.0f;
    jr[k][2] = cpt ? at(J2, gi) : 0.0f;
  }
  // 1/eps per x (loads in flight with the staging)
  for (int q = threadIdx.x; q < RX; q += TPB) {
    const int ai = a0x + q - H;
    const bool in = ai >= 0 && ai < Px;
    sieh[q] = in ? ieh[ai] : 1.0f;
    sien[q] = in ? ien[ai] : 1.0f;
  }
  __syncthreads();
  // ---- B: b^{n+1/2} on local [-2, T] (in place; reads E only)
  auto phase_b = [&](auto INNER) {
  for (int l = threadIdx.x; l < NR; l += TPB) {
    int qx, qy, qz;
    split(l, qx, qy, qz);
    if (qx > T::X + H || (D >= 2 && qy > T::Y + H) || (D >= 3 && qz > T::Z + H)) continue;
    const unsigned bx = INNER ? ~0u : sbx[qx], by = INNER ? ~0u : sby[qy], bz = INNER ? ~0u : sbz[qz];
    if ((bx & AX_BN) && (by & AX_BH) && (bz & AX_BH)) {
      float cu = 0.0f;
      if (D >= 2) cu += hy * (sE[2][l + LY] - sE[2][l]);
      if (D >= 3) cu -= hz * (sE[1][l + LZ] - sE[1][l]);
      sB[0][l] -= cu;
    }
    if ((bx & AX_BH) && (by & AX_BN) && (bz & AX_BH)) {
      float cu = -hx * (sE[2][l + 1] - sE[2][l]);
      if (D >= 3) cu += hz * (sE[0][l + LZ] - sE[0][l]);
      sB[1][l] -= cu;
    }
    if ((bx & AX_BH) && (by & AX_BH) && (bz & AX_BN)) {
      float cu = hx * (sE[1][l + 1] - sE[1][l]);
      if (D >= 2) cu -= hy * (sE[0][l + LY] - sE[0][l]);
      sB[2][l] -= cu;
    }
  }
  };
  if (inner) phase_b(std::true_type{});
  else phase_b(std::false_type{});
  __syncthreads();
  // ---- C: E^{n+1} at interior positions on local [-1, T] (in place)
  auto phase_c = [&](auto INNER) {
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    const int l = threadIdx.x + k * TPB;
    if (l >= NR) continue;
    int qx, qy, qz;
    split(l, qx, qy, qz);
    if (qx < H - 1 || qx > T::X + H) continue;
    if (D >= 2 && (qy < H - 1 || qy > T::Y + H)) continue;
    if (D >= 3 && (qz < H - 1 || qz > T::Z + H)) continue;
    const unsigned bx = INNER ? ~0u : sbx[qx], by = INNER ? ~0u : sby[qy], bz = INNER ? ~0u : sbz[qz];
    if (!INNER && !(bx & by & bz & AX_ARR)) continue;
    // Lorentz media: this block owns the position (periodic axes: the box)
    unsigned gl = 0u;
    bool own = false;
    float4 lh = make_float4(0.f, 0.f, 0.f, 0.f), ln = lh;   // oscillator coefficients at this x
    if (lorT) {
      const int ai = a0x + qx - H;
      if (ai >= 0 && ai < Px) {
        lh = I.lor_half[ai];
        ln = I.lor_node[ai];
      }
      gl = (unsigned)(ai + soy[qy] + soz[qz]);
      own = qx >= H && qx < T::X + H;
      if (D >= 2) own = own && qy >= H && qy < T::Y + H && (!py || (unsigned)(a0y + qy - H - Gy) < (unsigned)ny);
      if (D >= 3) own = own && qz >= H && qz < T::Z + H && (!pz || (unsigned)(a0z + qz - H - Gz) < (unsigned)nz);
    }
    if ((bx & AX_IH) && (by & AX_IN) && (bz & AX_IN)) {
      float cu = 0.0f;
      if (D >= 2) cu += Cy * (sB[2][l] - sB[2][l - LY]);
      if (D >= 3) cu -= Cz * (sB[1][l] - sB[1][l - LZ]);
      float src = cu - jr[k][0];
      if (lorT && lh.y != 0.0f) src -= lor_step(LOR_PTRS(I, par, 0), gl, lh, sE[0][l], own);
      if (LOR == 2 && lorT && lh.w != 0.0f)
        sE[0][l] = kerr_update(sE[0][l], sieh[qx], src, lh.w);
      else
        sE[0][l] += sieh[qx] * src;
    }
    if ((bx & AX_IN) && (by & AX_IH) && (bz & AX_IN)) {
      float cu = -Cx * (sB[2][l] - sB[2][l - 1]);
      if (D >= 3) cu += Cz * (sB[0][l] - sB[0][l - LZ]);
      float src = cu - jr[k][1];
      if (lorT && ln.y != 0.0f) src -= lor_step(LOR_PTRS(I, par, 1), gl, ln, sE[1][l], own);
      if (LOR == 2 && lorT && ln.w != 0.0f)
        sE[1][l] = kerr_update(sE[1][l], sien[qx], src, ln.w);
      else
        sE[1][l] += sien[qx] * src;
    }
    if ((bx & AX_IN) && (by & AX_IN) && (bz & AX_IH)) {
      float cu = Cx * (sB[1][l] - sB[1][l - 1]);
      if (D >= 2) cu -= Cy * (sB[0][l] - sB[0][l - LY]);
      float src = cu - jr[k][2];
      if (lorT && ln.y != 0.0f) src -= lor_step(LOR_PTRS(I, par, 2), gl, ln, sE[2][l], own);
      if (LOR == 2 && lorT && ln.w != 0.0f)
        sE[2][l] = kerr_update(sE[2][l], sien[qx], src, ln.w);
      else
        sE[2][l] += sien[qx] * src;
    }
  }
  };
  if (inner) phase_c(std::true_type{});
  else phase_c(std::false_type{});
  __syncthreads();
  // ---- D: outflow faces, lowest priority first (z, y, x); a point on several
  // faces follows the first of x, y, z, with its inward neighbour's final value
#pragma unroll
  for (int d = 2; d >= 0; --d) {
    if (d >= D) continue;
    const bool perd = d == 1 ? py : (d == 2 ? pz : false);
    if (perd) continue;
    const int nd = d == 0 ? nx : (d == 1 ? ny : nz);
    const int o0 = d == 0 ? i0 : (d == 1 ? j0 : k0);
    const int Td = d == 0 ? T::X : (d == 1 ? T::Y : T::Z);
    // does the tile's E region [-1, T] along d touch a face?
    const bool touch = (o0 - 1 <= 0 && 0 <= o0 + Td) || (o0 - 1 <= nd && nd <= o0 + Td);
    if (touch) {
      const int ls = d == 0 ? 1 : (d == 1 ? LY : LZ);
      float4 s0 = make_float4(0.f, 0.f, 0.f, 0.f), s1 = s0;
      if (d == 0) {
        if (step < I.nsrc) s0 = I.src[step];
        if (step + 1 < I.nsrc) s1 = I.src[step + 1];
      }
      for (int l = threadIdx.x; l < NR; l += TPB) {
        int qx, qy, qz;
        split(l, qx, qy, qz);
        if (qx < H - 1 || qx > T::X + H) continue;
        if (D >= 2 && (qy < H - 1 || qy > T::Y + H)) continue;
        if (D >= 3 && (qz < H - 1 || qz > T::Z + H)) continue;
        const unsigned bx = sbx[qx], by = sby[qy], bz = sbz[qz];
        const unsigned bd = d == 0 ? bx : (d == 1 ? by : bz);
        if (!(bd & (AX_F0 | AX_F1))) continue;
        const int inw = (bd & AX_F0) ? 1 : -1;
        const int qd = (d == 0 ? qx : (d == 1 ? qy : qz)) + inw;
        if (qd < H - 1 || qd > Td + H) continue;
        const unsigned bb[3] = {bx, by, bz};
        const unsigned gq = (unsigned)(a0x + qx - H + soy[qy] + soz[qz]);
        const unsigned gr = gq + (d == 0 ? inw : (d == 1 ? inw * sy : inw * sz));
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (c == d) continue;   // normal component: interior update only
          // inside the box along the other axes, not on a face of higher priority
          bool ok = true;
#pragma unroll
          for (int e = 0; e < 3; ++e) {
            if (e == d || e >= D) continue;
            const bool half = (e == c);
            if (e < d) ok = ok && (bb[e] & (half ? AX_IH : AX_IN));
            else ok = ok && (bb[e] & (half ? AX_BH : AX_BN));   // box incl. faces (periodic: any)
          }
          if (!ok) continue;
          const gmem<float>* Eold = c == 0 ? Ec0 : (c == 1 ? Ec1 : Ec2);
          const float qold = at(Eold, gq), rold = at(Eold, gr), rnew = sE[c][l + inw * ls];
          if (d == 0 && (bd & AX_F0) && c == I.pol) {
            const float pr = I.prof[(soy[qy] / sy) + Py * (D >= 3 ? soz[qz] / sz : 0)];
            const MurInc m{pr * s0.x, pr * s1.x, pr * s0.y, pr * s1.y};
            sE[c][l] = mur_inc(qold, rold, rnew, I.kmur[0], m);
          } else {
            sE[c][l] = mur(qold, rold, rnew, I.kmur[d]);
          }
        }
      }
    }
    __syncthreads();
  }
  // ---- E: owned positions: b^{n+1}, E^{n+1} out, J cleared, amplitude window,
  // the Poynting flux through the planes one node inside the outflow faces
  auto hits = [](int lo, int t, int p) { return p >= lo && p < lo + t; };
  bool flux_tile = hits(a0x, T::X, G + 1) || hits(a0x, T::X, G + nx - 1);
  if (D >= 2 && !py) flux_tile = flux_tile || hits(a0y, T::Y, G + 1) || hits(a0y, T::Y, G + ny - 1);
  if (D >= 3 && !pz) flux_tile = flux_tile || hits(a0z, T::Z, G + 1) || hits(a0z, T::Z, G + nz - 1);
  double fin = 0.0, fout = 0.0;   // this thread's energy into / out of the inner box
  float chk = 0.0f;               // NaN once a stored E is not finite
  const int nwin = I.nwin;
  const int slot = step % (nwin > 0 ? nwin : 1);
  const int wx0 = I.wx0, wx1 = I.wx1;
  bool stored_nz = false;   // this thread stored a nonzero E or b (tiles reaching past the front)
  const bool track = a0x + T::X - 1 > front;
  auto phase_e = [&](auto INNER) {
  for (int l = threadIdx.x; l < NR; l += TPB) {
    int qx, qy, qz;
    split(l, qx, qy, qz);
    if (qx < H || qx >= T::X + H) continue;
    if (D >= 2 && (qy < H || qy >= T::Y + H)) continue;
    if (D >= 3 && (qz < H || qz >= T::Z + H)) continue;
    const int ai = a0x + qx - H;
    const int aj = D >= 2 ? a0y + qy - H : 0;   // absent axes: index 0
    const int ak = D >= 3 ? a0z + qz - H : 0;
    if (!INNER && (ai >= Px || aj >= Py || ak >= Pz)) continue;
    const unsigned gi = (unsigned)(ai + sy * aj + sz * ak);
    if (cur) {
      at(Jn0, gi) = 0.0f;   // next push deposits here; nobody reads it now
      at(Jn1, gi) = 0.0f;
      at(Jn2, gi) = 0.0f;
    }
    const unsigned bx = INNER ? ~0u : sbx[qx], by = INNER ? ~0u : sby[qy], bz = INNER ? ~0u : sbz[qz];
    // owned positions of periodic axes are the box itself (no wrapped copies)
    const unsigned dy = !INNER && D >= 2 && py ? (aj - G >= 0 && aj - G < ny ? ~0u : 0u) : ~0u;
    const unsigned dz = !INNER && D >= 3 && pz ? (ak - G >= 0 && ak - G < nz ? ~0u : 0u) : ~0u;
    const bool xdn = bx & AX_DN, xdh = bx & AX_DH;
    const bool ydn = by & dy & AX_DN, ydh = by & dy & AX_DH;
    const bool zdn = bz & dz & AX_DN, zdh = bz & dz & AX_DH;
    if (xdh && ydn && zdn) {
      at(En0, gi) = sE[0][l];
      stored_nz = stored_nz || (track && sE[0][l] != 0.0f);
    }
    if (xdn && ydh && zdn) {
      at(En1, gi) = sE[1][l];
      stored_nz = stored_nz || (track && sE[1][l] != 0.0f);
    }
    if (xdn && ydn && zdh) {
      at(En2, gi) = sE[2][l];
      stored_nz = stored_nz || (track && sE[2][l] != 0.0f);
    }
    // non-finite E (a NaN or an infinity anywhere in the sum leaves chk NaN)
    chk = fmaf(sE[0][l] + sE[1][l] + sE[2][l], 0.0f, chk);
    if (flux_tile) {
      const int i = ai - G, j = D >= 2 ? aj - G : 0, k = D >= 3 ? ak - G : 0;
      // trapezoid weights of the inner box [1, n - 1] along a transverse axis:
      // node positions (ends 1/2), half-staggered positions (1 <= v <= n - 2);
      // periodic and absent axes weigh every (owned) position 1
      auto wn = [](int v, int n, bool per) -> double {
        if (per) return 1.0;
        if (v < 1 || v > n - 1) return 0.0;
        return (v == 1 || v == n - 1) ? 0.5 : 1.0;
      };
      auto wh = [](int v, int n, bool per) -> double { return per || (v >= 1 && v <= n - 2) ? 1.0 : 0.0; };
      const bool ay = D < 2 || py, az = D < 3 || pz;   // y, z weigh 1
      // one product E_a (at the half step) b_b (averaged to the plane along d)
      auto term = [&](double w, float en, float eo, float b0, float b1, double coef) {
        if (w == 0.0) return;
        const double v = coef * w * (0.5 * ((double)en + (double)eo)) * (0.5 * ((double)b0 + (double)b1));
        if (v > 0.0) fin += v; else fout -= v;
      };
      // plane normal to x: S_x = E_y b_z - E_z b_y
      if (xdn && (i == 1 || i == nx - 1)) {
        const double c = (i == 1 ? 1.0 : -1.0) * I.kflux[0];
        if (ydh && zdn) term(wh(j, ny, ay) * wn(k, nz, az), sE[1][l], at(Ec1, gi), sB[2][l - 1], sB[2][l], c);
        if (ydn && zdh) term(wn(j, ny, ay) * wh(k, nz, az), sE[2][l], at(Ec2, gi), sB[1][l - 1], sB[1][l], -c);
      }
      // plane normal to y: S_y = E_z b_x - E_x b_z
      if (D >= 2 && !py && ydn && (j == 1 || j == ny - 1)) {
        const double c = (j == 1 ? 1.0 : -1.0) * I.kflux[1];
        if (xdn && zdh) term(wn(i, nx, false) * wh(k, nz, az), sE[2][l], at(Ec2, gi), sB[0][l - LY], sB[0][l], c);
        if (xdh && zdn) term(wh(i, nx, false) * wn(k, nz, az), sE[0][l], at(Ec0, gi), sB[2][l - LY], sB[2][l], -c);
      }
      // plane normal to z: S_z = E_x b_y - E_y b_x
      if (D >= 3 && !pz && zdn && (k == 1 || k == nz - 1)) {
        const double c = (k == 1 ? 1.0 : -1.0) * I.kflux[2];
        if (xdh && ydn) term(wh(i, nx, false) * wn(j, ny, py), sE[0][l], at(Ec0, gi), sB[1][l - LZ], sB[1][l], c);
        if (xdn && ydh) term(wn(i, nx, false) * wh(j, ny, py), sE[1][l], at(Ec1, gi), sB[0][l - LZ], sB[0][l], -c);
      }
    }
    if (xdn && ydh && zdh) {
      float cu = 0.0f;
      if (D >= 2) cu += hy * (sE[2][l + LY] - sE[2][l]);
      if (D >= 3) cu -= hz * (sE[1][l + LZ] - sE[1][l]);
      const float v = sB[0][l] - cu;
      at(Bn0, gi) = v;
      stored_nz = stored_nz || (track && v != 0.0f);
    }
    if (xdh && ydn && zdh) {
      float cu = -hx * (sE[2][l + 1] - sE[2][l]);
      if (D >= 3) cu += hz * (sE[0][l + LZ] - sE[0][l]);
      const float v = sB[1][l] - cu;
      at(Bn1, gi) = v;
      stored_nz = stored_nz || (track && v != 0.0f);
    }
    if (xdh && ydh && zdn) {
      float cu = hx * (sE[1][l + 1] - sE[1][l]);
      if (D >= 2) cu -= hy * (sE[0][l + LY] - sE[0][l]);
      const float v = sB[2][l] - cu;
      at(Bn2, gi) = v;
      stored_nz = stored_nz || (track && v != 0.0f);
    }
    // node |E^{n+1}| (Yee components averaged to the node) into the window
    if (ai >= wx0 && ai < wx1 && xdn && ydn && zdn) {
      const float ex = 0.5f * (sE[0][l - 1] + sE[0][l]);
      const float ey = D >= 2 ? 0.5f * (sE[1][l - LY] + sE[1][l]) : sE[1][l];
      const float ez = D >= 3 ? 0.5f * (sE[2][l - LZ] + sE[2][l]) : sE[2][l];
      const float m = sqrtf(ex * ex + ey * ey + ez * ez);
      if (!(m <= 3.0e38f)) atomicOr(I.health, HEALTH_NONFINITE);
      const int64_t wsz = I.wsz;
      const int64_t w = (int64_t)(ai - wx0) + (int64_t)I.wnx * (aj + (int64_t)Py * ak);
      gmem<float>* __restrict__ ring = gp(I.ring);
      gmem<float>* __restrict__ suffix = gp(I.suffix);
      ring[(int64_t)slot * wsz + w] = m;
      gmem<float>* __restrict__ prefix = gp(I.prefix);
      const float pre = slot == 0 ? m : fmaxf(prefix[w], m);
      prefix[w] = pre;
      const float a = slot + 1 < nwin ? fmaxf(suffix[(int64_t)(slot + 1) * wsz + w], pre) : pre;
      at(gp(uniform(I.A)), gi) = a;
      if (a >= I.acut_min) blk_hot = 1;
      if (!ONE && slot == nwin - 1) {   // block of samples complete: suffix maxima for the next
        // (a single run rebuilds them in k_win_rebuild, all nodes in parallel)
        float run = 0.0f;
        for (int q = nwin - 1; q >= 0; --q) {
          run = fmaxf(run, ring[(int64_t)q * wsz + w]);
          suffix[(int64_t)q * wsz + w] = run;
        }
      }
    }
  }
  };
  if (inner) phase_e(std::true_type{});
  else phase_e(std::false_type{});
  // a tile reaching past the field front moves it if it stored a nonzero value
  if (track) {
    if (__syncthreads_or(stored_nz) && threadIdx.x == 0) atomicMax(frontp, a0x + T::X - 1);
  } else {
    __syncthreads();
  }
  if (threadIdx.x == 0 && blk_hot) atomicOr(I.hot + par, 1);
  if (threadIdx.x == 0) atomicAdd(I.tiles_done + 32 * (blockIdx.x & 7), 1ull);
  if (chk != 0.0f) atomicOr(I.health, HEALTH_NONFINITE);
  if (flux_tile) {
    for (int o = 32; o > 0; o >>= 1) {
      fin += __shfl_xor(fin, o);
      fout += __shfl_xor(fout, o);
    }
    if ((threadIdx.x & 63) == 0) {
      double* ef = I.eflux + (blockIdx.x & 7) * 32;   // this XCD's line
      if (fin != 0.0) atomicAdd(ef, fin);
      if (fout != 0.0) atomicAdd(ef + 1, fout);
    }
  }
}

// ------------------------------------------------- field update, z-marching
// The 3D update for periodic y and z as a march along z: a block owns an x-y
// tile of ZX x ZY positions (x over the padded array, y over the box) and a
// segment of ZS planes, and walks its planes upward with the halo of the
// tiled update in x and y only (64 x 12 staged points per plane, 1.6x the
// owned ones, against 5.3x for a 12 x 4 x 4 tile).  The launch's block count
// sets the number of z segments.  Each thread keeps three
// points of the plane; the next plane's fields and current are loaded while
// the current plane is computed.  Plane t of the march: b^{n+1/2}(t) from
// E^n(t) (in-plane neighbours, LDS) and E^n(t+1) (own point, registers);
// E^{n+1}(t) from b^{n+1/2}(t) (LDS) and b^{n+1/2}(t-1) (registers); the x
// faces of plane t; then plane t-1 is finished: b^{n+1}, the stores, the
// current cleared, the amplitude window and the Poynting flux.  Every
// position gets the same arithmetic as in the tiled update.
constexpr int ZX = 60, ZY = 8, ZH = 2;
constexpr int ZRX = ZX + 2 * ZH, ZRY = ZY + 2 * ZH;   // 64 x 12 staged
constexpr int ZNP = ZRX * ZRY;
constexpr int ZPT = ZNP / TPB;                        // points per thread
static_assert(ZNP % TPB == 0 && ZRX == 64, "plane layout");

template <bool ONE, int LOR>
__global__ __launch_bounds__(TPB, 4) void k_fields_z(Group g, std::conditional_t<ONE, Inst, NoInst> one) {
  constexpr int LY = ZRX;
  __shared__ float sEa[3][ZNP], sEb[3][ZNP], sBa[3][ZNP], sBb[3][ZNP];
  // E^n_y, E^n_z of the last two planes at the x-face columns [side][0] and
  // their inward neighbours [side][1] (the Mur conditions' old values; the
  // inward columns are also the flux planes), kept before E^{n+1} overwrites
  __shared__ float sOld[2][2][2][2][ZRY];
  __shared__ unsigned sbx[ZRX];
  __shared__ float sieh[ZRX], sien[ZRX];
  __shared__ float4 slh[LOR ? ZRX : 1], sln[LOR ? ZRX : 1];   // Lorentz coefficients per x
  __shared__ int blk_hot;
  const Slot sl = ONE ? Slot{0, (int)blockIdx.x, g.blocks} : block_slot(g);
  auto& I = inst_of(g, sl.ii, one);
  const int step = ONE || g.step >= 0 ? g.step : I.step_now;
  const int par = step & 1;
  int* const frontp = ONE ? g.front : I.front;
  gmem<int>* const xe = gp(const_cast<int*>(ONE ? g.xext : I.xext) + 2 * (step % 3));
  const int front = __hip_atomic_load(gp(frontp), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  const int xlo = __hip_atomic_load(xe, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  const int xhi = __hip_atomic_load(xe + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  const gmem<float>* __restrict__ Ec0 = gp(uniform(I.F[par][0]));
  const gmem<float>* __restrict__ Ec1 = gp(uniform(I.F[par][1]));
  const gmem<float>* __restrict__ Ec2 = gp(uniform(I.F[par][2]));
  const gmem<float>* __restrict__ Bc0 = gp(uniform(I.F[par][3]));
  const gmem<float>* __restrict__ Bc1 = gp(uniform(I.F[par][4]));
  const gmem<float>* __restrict__ Bc2 = gp(uniform(I.F[par][5]));
  gmem<float>* __restrict__ En0 = gp(uniform(I.F[par ^ 1][0]));
  gmem<float>* __restrict__ En1 = gp(uniform(I.F[par ^ 1][1]));
  gmem<float>* __restrict__ En2 = gp(uniform(I.F[par ^ 1][2]));
  gmem<float>* __restrict__ Bn0 = gp(uniform(I.F[par ^ 1][3]));
  gmem<float>* __restrict__ Bn1 = gp(uniform(I.F[par ^ 1][4]));
  gmem<float>* __restrict__ Bn2 = gp(uniform(I.F[par ^ 1][5]));
  const gmem<float>* __restrict__ J0 = gp(uniform(I.Jb[par][0]));
  const gmem<float>* __restrict__ J1 = gp(uniform(I.Jb[par][1]));
  const gmem<float>* __restrict__ J2 = gp(uniform(I.Jb[par][2]));
  gmem<float>* __restrict__ Jn0 = gp(uniform(I.Jb[par ^ 1][0]));
  gmem<float>* __restrict__ Jn1 = gp(uniform(I.Jb[par ^ 1][1]));
  gmem<float>* __restrict__ Jn2 = gp(uniform(I.Jb[par ^ 1][2]));
  const float hx = I.halfC[0], hy = I.halfC[1], hz = I.halfC[2];
  const float Cx = I.C[0], Cy = I.C[1], Cz = I.C[2];
  const int Px = I.Px, Py = I.Py;
  const int nx = I.nx, ny = I.ny, nz = I.nz;
  const int sy = I.sy, sz = I.sz, Gy = I.Gy, Gz = I.Gz;
  const int ntx = (Px + ZX - 1) / ZX, nty = (ny + ZY - 1) / ZY;
  const int tb = xcd_remap(sl.bk, sl.nbk);
  const int tx = tb % ntx, rest = tb / ntx;
  const int ty = rest % nty, seg = rest / nty;
  const int nseg = sl.nbk / (ntx * nty);   // segments of z (the launch's block count decides)
  const int zs = (nz + nseg - 1) / nseg;
  const int a0x = tx * ZX;           // padded x of local column ZH
  const int j0 = ty * ZY;            // y of local row ZH
  const int k0 = seg * zs, k1 = min(k0 + zs, nz);
  // far tiles (no current ever) and tiles beyond the field front, as in the tiled update
  bool cur = true;
  if (g.part >= 1) {
    int lo = xlo, hi = xhi;
    if (I.wx1 > I.wx0) {
      lo = min(lo, I.wx0 - G);
      hi = max(hi, I.wx1 - 1 - G);
    }
    const int alo = lo - XNEAR_MARGIN + G, ahi = hi + XNEAR_MARGIN + G;
    cur = lo <= hi && a0x <= ahi && a0x + ZX - 1 >= alo;
  }
  if (g.part == 1 && !cur && a0x - ZH > front) return;
  if (threadIdx.x == 0) blk_hot = 0;
  const bool lorT = LOR && I.lx0 < I.lx1 && a0x - ZH < I.lx1 && a0x + ZX + ZH > I.lx0;
  for (int q = threadIdx.x; q < ZRX; q += TPB) {
    const int i = a0x - G + q - ZH;
    const int ai = a0x + q - ZH;
    sbx[q] = axis_bits(i, nx, false, ai >= 0 && ai < Px);
    const bool in = ai >= 0 && ai < Px;
    sieh[q] = in ? I.ie_half[ai] : 1.0f;
    sien[q] = in ? I.ie_node[ai] : 1.0f;
    if (lorT) {
      slh[q] = in ? I.lor_half[ai] : make_float4(0.f, 0.f, 0.f, 0.f);
      sln[q] = in ? I.lor_node[ai] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  // this thread's points: row offsets (y wrapped) and per-point facts
  int qxs[ZPT], qys[ZPT];
  unsigned rowo[ZPT];
  bool owny[ZPT];
#pragma unroll
  for (int p = 0; p < ZPT; ++p) {
    const int l = threadIdx.x + p * TPB;
    qxs[p] = l & (ZRX - 1);
    qys[p] = l / ZRX;
    const int j = j0 + qys[p] - ZH;
    rowo[p] = (unsigned)(sy * (wrap_any(j, ny) + Gy));
    owny[p] = qys[p] >= ZH && qys[p] < ZH + ZY && j < ny;
  }
  __syncthreads();
  auto plane = [&](int k) { return (unsigned)(sz * (wrap_any(k, nz) + Gz)); };
  auto pt_in = [&](int p) { return (sbx[qxs[p]] & AX_ARR) != 0u; };
  auto eregion = [&](int p) {
    return qxs[p] >= ZH - 1 && qxs[p] <= ZX + ZH && qys[p] >= ZH - 1 && qys[p] <= ZY + ZH;
  };
  // loads of plane k: E^n and b^n at every staged point, J at the E region
  auto load_eb = [&](int k, float (&e)[ZPT][3], float (&b)[ZPT][3]) {
    const unsigned pk = plane(k);
#pragma unroll
    for (int p = 0; p < ZPT; ++p) {
      const bool in = pt_in(p);
      const unsigned gi = (unsigned)(a0x + qxs[p] - ZH) + rowo[p] + pk;
      e[p][0] = in ? at(Ec0, gi) : 0.0f;
      e[p][1] = in ? at(Ec1, gi) : 0.0f;
      e[p][2] = in ? at(Ec2, gi) : 0.0f;
      b[p][0] = in ? at(Bc0, gi) : 0.0f;
      b[p][1] = in ? at(Bc1, gi) : 0.0f;
      b[p][2] = in ? at(Bc2, gi) : 0.0f;
    }
  };
  auto load_j = [&](int k, float (&j)[ZPT][3]) {
    const unsigned pk = plane(k);
#pragma unroll
    for (int p = 0; p < ZPT; ++p) {
      const bool c = cur && pt_in(p) && eregion(p);
      const unsigned gi = (unsigned)(a0x + qxs[p] - ZH) + rowo[p] + pk;
      j[p][0] = c ? at(J0, gi) : 0.0f;
      j[p][1] = c ? at(J1, gi) : 0.0f;
      j[p][2] = c ? at(J2, gi) : 0.0f;
    }
  };
  // plane buffers: c* the plane being advanced, p* the plane before it
  float (*cE)[ZNP] = sEa;
  float (*pE)[ZNP] = sEb;
  float (*cB)[ZNP] = sBa;
  float (*pB)[ZNP] = sBb;
  float ne[ZPT][3], nb[ZPT][3];     // E^n, b^n of plane t + 1
  float ne2[ZPT][3], nb2[ZPT][3];   // of plane t + 2 (in flight)
  float jc[ZPT][3], jn[ZPT][3];     // J of plane t, t + 1
  float bh0[ZPT], bh1[ZPT];         // b^{n+1/2}_x, _y of plane t - 1 at the own points
  float e2p[ZPT], e2pp[ZPT];        // final E_z of planes t - 1, t - 2
  {
    float e0[ZPT][3], b0[ZPT][3];
    load_eb(k0 - 2, e0, b0);
    load_eb(k0 - 1, ne, nb);
    load_j(k0 - 2, jc);
#pragma unroll
    for (int p = 0; p < ZPT; ++p) {
      const int l = threadIdx.x + p * TPB;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        cE[c][l] = e0[p][c];
        cB[c][l] = b0[p][c];
      }
      bh0[p] = bh1[p] = e2p[p] = e2pp[p] = 0.0f;
    }
  }
  __syncthreads();
  const bool xface = (a0x - G - ZH + 1 <= 0 && 0 <= a0x - G + ZX) || (a0x - G - ZH + 1 <= nx && nx <= a0x - G + ZX);
  const bool flux_tile = (a0x <= G + 1 && G + 1 < a0x + ZX) || (a0x <= G + nx - 1 && G + nx - 1 < a0x + ZX);
  const bool track = a0x + ZX - 1 > front;
  gmem<float>* __restrict__ wring = gp(I.ring);
  gmem<float>* __restrict__ wprefix = gp(I.prefix);
  gmem<float>* __restrict__ wsuffix = gp(I.suffix);
  const int nwin = I.nwin;
  const int slot = step % (nwin > 0 ? nwin : 1);
  const int wx0 = I.wx0, wx1 = I.wx1;
  double fin = 0.0, fout = 0.0;
  float chk = 0.0f;
  bool stored_nz = false;
  float4 s0 = make_float4(0.f, 0.f, 0.f, 0.f), s1 = s0;
  if (step < I.nsrc) s0 = I.src[step];
  if (step + 1 < I.nsrc) s1 = I.src[step + 1];
  for (int t = k0 - 2; t <= k1 && k0 < k1; ++t) {
    load_eb(t + 2, ne2, nb2);
    load_j(t + 1, jn);
    // ---- b^{n+1/2}(t) on local [-2, T] (in place)
#pragma unroll
    for (int p = 0; p < ZPT; ++p) {
      const int l = threadIdx.x + p * TPB;
      const int qx = qxs[p], qy = qys[p];
      if (qx > ZX + ZH || qy > ZY + ZH) continue;
      const unsigned bx = sbx[qx];
      if (bx & AX_BN) {
        float cu = 0.0f;
        cu += hy * (cE[2][l + LY] - cE[2][l]);
        cu -= hz * (ne[p][1] - cE[1][l]);
        cB[0][l] -= cu;
      }
      if (bx & AX_BH) {
        float cu = -hx * (cE[2][l + 1] - cE[2][l]);
        cu += hz * (ne[p][0] - cE[0][l]);
        cB[1][l] -= cu;
      }
      if (bx & AX_BH) {
        float cu = hx * (cE[1][l + 1] - cE[1][l]);
        cu -= hy * (cE[0][l + LY] - cE[0][l]);
        cB[2][l] -= cu;
      }
    }
    if (xface) {
#pragma unroll
      for (int p = 0; p < ZPT; ++p) {
        const int l = threadIdx.x + p * TPB;
        const int qx = qxs[p], qy = qys[p];
        const unsigned bx = sbx[qx];
        int side = -1, fi = 0;
        if (bx & AX_F0) side = 0;
        else if (bx & AX_F1) side = 1;
        else if (qx >= 1 && (sbx[qx - 1] & AX_F0)) side = 0, fi = 1;
        else if (qx + 1 < ZRX && (sbx[qx + 1] & AX_F1)) side = 1, fi = 1;
        if (side >= 0) {
          sOld[t & 1][side][fi][0][qy] = cE[1][l];
          sOld[t & 1][side][fi][1][qy] = cE[2][l];
        }
      }
    }
    __syncthreads();
    if (t >= k0 - 1) {
      // ---- E^{n+1}(t) on local [-1, T] (in place)
#pragma unroll
      for (int p = 0; p < ZPT; ++p) {
        const int l = threadIdx.x + p * TPB;
        const int qx = qxs[p];
        if (!eregion(p)) continue;
        const unsigned bx = sbx[qx];
        if (!(bx & AX_ARR)) continue;
        // Lorentz media: this block owns the position (plane t of its segment)
        unsigned gl = 0u;
        bool own = false;
        if (lorT) {
          gl = (unsigned)(a0x + qx - ZH) + rowo[p] + plane(t);
          own = qx >= ZH && qx < ZX + ZH && owny[p] && t >= k0 && t < k1;
        }
        if (bx & AX_IH) {
          float cu = 0.0f;
          cu += Cy * (cB[2][l] - cB[2][l - LY]);
          cu -= Cz * (cB[1][l] - bh1[p]);
          float src = cu - jc[p][0];
          if (lorT && slh[qx].y != 0.0f) src -= lor_step(LOR_PTRS(I, par, 0), gl, slh[qx], cE[0][l], own);
          if (LOR == 2 && lorT && slh[qx].w != 0.0f)
            cE[0][l] = kerr_update(cE[0][l], sieh[qx], src, slh[qx].w);
          else
            cE[0][l] += sieh[qx] * src;
        }
        if (bx & AX_IN) {
          float cu = -Cx * (cB[2][l] - cB[2][l - 1]);
          cu += Cz * (cB[0][l] - bh0[p]);
          float src = cu - jc[p][1];
          if (lorT && sln[qx].y != 0.0f) src -= lor_step(LOR_PTRS(I, par, 1), gl, sln[qx], cE[1][l], own);
          if (LOR == 2 && lorT && sln[qx].w != 0.0f)
            cE[1][l] = kerr_update(cE[1][l], sien[qx], src, sln[qx].w);
          else
            cE[1][l] += sien[qx] * src;
        }
        if (bx & AX_IN) {
          float cu = Cx * (cB[1][l] - cB[1][l - 1]);
          cu -= Cy * (cB[0][l] - cB[0][l - LY]);
          float src = cu - jc[p][2];
          if (lorT && sln[qx].y != 0.0f) src -= lor_step(LOR_PTRS(I, par, 2), gl, sln[qx], cE[2][l], own);
          if (LOR == 2 && lorT && sln[qx].w != 0.0f)
            cE[2][l] = kerr_update(cE[2][l], sien[qx], src, sln[qx].w);
          else
            cE[2][l] += sien[qx] * src;
        }
      }
      __syncthreads();
      // ---- x faces of plane t (y and z periodic: no other face)
      if (xface) {
        const unsigned pk = plane(t);
#pragma unroll
        for (int p = 0; p < ZPT; ++p) {
          const int l = threadIdx.x + p * TPB;
          const int qx = qxs[p];
          if (!eregion(p)) continue;
          const unsigned bx = sbx[qx];
          if (!(bx & (AX_F0 | AX_F1))) continue;
          const int inw = (bx & AX_F0) ? 1 : -1;
          const int qd = qx + inw;
          if (qd < ZH - 1 || qd > ZX + ZH) continue;
          const int side = (bx & AX_F0) ? 0 : 1;
#pragma unroll
          for (int c = 1; c < 3; ++c) {
            const float qold = sOld[t & 1][side][0][c - 1][qys[p]], rold = sOld[t & 1][side][1][c - 1][qys[p]];
            const float rnew = cE[c][l + inw];
            if ((bx & AX_F0) && c == I.pol) {
              const float pr = I.prof[(int)(rowo[p] / (unsigned)sy) + Py * (int)(pk / (unsigned)sz)];
              const MurInc m{pr * s0.x, pr * s1.x, pr * s0.y, pr * s1.y};
              cE[c][l] = mur_inc(qold, rold, rnew, I.kmur[0], m);
            } else {
              cE[c][l] = mur(qold, rold, rnew, I.kmur[0]);
            }
          }
        }
        // no barrier: a face value is read next by its own thread (b^{n+1}
        // of plane t - 1 below), by the others only after the rotation's
      }
    }
    // ---- finish plane f = t - 1 at the owned positions: first the loads
    // it needs (window samples, old E on the flux planes), in flight while
    // the fields are stored
    if (t >= k0 + 1) {
      const int f = t - 1;
      const unsigned pk = plane(f);
      const int ak = wrap_any(f, nz) + Gz;   // padded z of plane f
      const int64_t wsz = I.wsz;
      float wpre[ZPT], wsuf[ZPT], eo1[ZPT], eo2[ZPT];
      int64_t wix[ZPT];
#pragma unroll
      for (int p = 0; p < ZPT; ++p) {
        wpre[p] = wsuf[p] = eo1[p] = eo2[p] = 0.0f;
        wix[p] = -1;
        const int qx = qxs[p];
        if (qx < ZH || qx >= ZX + ZH || !owny[p]) continue;
        const int ai = a0x + qx - ZH;
        if (ai >= Px) continue;
        const unsigned gi = (unsigned)ai + rowo[p] + pk;
        const unsigned bx = sbx[qx];
        if (ai >= wx0 && ai < wx1 && (bx & AX_DN)) {
          const int aj = (int)(rowo[p] / (unsigned)sy);
          const int64_t w = (int64_t)(ai - wx0) + (int64_t)I.wnx * (aj + (int64_t)Py * ak);
          wix[p] = w;
          if (slot != 0) wpre[p] = wprefix[w];
          if (slot + 1 < nwin) wsuf[p] = wsuffix[(int64_t)(slot + 1) * wsz + w];
        }
        const int i = ai - G;
        if (flux_tile && (bx & AX_DN) && (i == 1 || i == nx - 1)) {
          // the flux planes are the columns next to the x faces
          const int side = i == 1 ? 0 : 1;
          eo1[p] = sOld[f & 1][side][1][0][qys[p]];
          eo2[p] = sOld[f & 1][side][1][1][qys[p]];
        }
      }
#pragma unroll
      for (int p = 0; p < ZPT; ++p) {
        const int l = threadIdx.x + p * TPB;
        const int qx = qxs[p];
        if (qx < ZH || qx >= ZX + ZH || !owny[p]) continue;
        const int ai = a0x + qx - ZH;
        if (ai >= Px) continue;
        const unsigned gi = (unsigned)ai + rowo[p] + pk;
        if (cur) {
          at(Jn0, gi) = 0.0f;
          at(Jn1, gi) = 0.0f;
          at(Jn2, gi) = 0.0f;
        }
        const unsigned bx = sbx[qx];
        const bool xdn = bx & AX_DN, xdh = bx & AX_DH;
        if (xdh) {
          at(En0, gi) = pE[0][l];
          stored_nz = stored_nz || (track && pE[0][l] != 0.0f);
        }
        if (xdn) {
          at(En1, gi) = pE[1][l];
          stored_nz = stored_nz || (track && pE[1][l] != 0.0f);
          at(En2, gi) = pE[2][l];
          stored_nz = stored_nz || (track && pE[2][l] != 0.0f);
        }
        chk = fmaf(pE[0][l] + pE[1][l] + pE[2][l], 0.0f, chk);
        if (flux_tile) {
          const int i = ai - G;
          auto term = [&](float en, float eo, float b0v, float b1v, double coef) {
            const double v = coef * 1.0 * (0.5 * ((double)en + (double)eo)) * (0.5 * ((double)b0v + (double)b1v));
            if (v > 0.0) fin += v; else fout -= v;
          };
          if (xdn && (i == 1 || i == nx - 1)) {
            const double c = (i == 1 ? 1.0 : -1.0) * I.kflux[0];
            term(pE[1][l], eo1[p], pB[2][l - 1], pB[2][l], c);
            term(pE[2][l], eo2[p], pB[1][l - 1], pB[1][l], -c);
          }
        }
        if (xdn) {
          float cu = 0.0f;
          cu += hy * (pE[2][l + LY] - pE[2][l]);
          cu -= hz * (cE[1][l] - pE[1][l]);
          const float v = pB[0][l] - cu;
          at(Bn0, gi) = v;
          stored_nz = stored_nz || (track && v != 0.0f);
        }
        if (xdh) {
          float cu = -hx * (pE[2][l + 1] - pE[2][l]);
          cu += hz * (cE[0][l] - pE[0][l]);
          const float v = pB[1][l] - cu;
          at(Bn1, gi) = v;
          stored_nz = stored_nz || (track && v != 0.0f);
          float cu2 = hx * (pE[1][l + 1] - pE[1][l]);
          cu2 -= hy * (pE[0][l + LY] - pE[0][l]);
          const float v2 = pB[2][l] - cu2;
          at(Bn2, gi) = v2;
          stored_nz = stored_nz || (track && v2 != 0.0f);
        }
        if (wix[p] >= 0) {
          const int64_t w = wix[p];
          const float ex = 0.5f * (pE[0][l - 1] + pE[0][l]);
          const float ey = 0.5f * (pE[1][l - LY] + pE[1][l]);
          const float ez = 0.5f * (e2pp[p] + pE[2][l]);
          const float m = sqrtf(ex * ex + ey * ey + ez * ez);
          if (!(m <= 3.0e38f)) atomicOr(I.health, HEALTH_NONFINITE);
          wring[(int64_t)slot * wsz + w] = m;
          const float pre = slot == 0 ? m : fmaxf(wpre[p], m);
          wprefix[w] = pre;
          const float a = slot + 1 < nwin ? fmaxf(wsuf[p], pre) : pre;
          at(gp(uniform(I.A)), gi) = a;
          if (a >= I.acut_min) blk_hot = 1;
          if (!ONE && slot == nwin - 1) {   // (single runs: k_win_rebuild)
            float run = 0.0f;
            for (int q = nwin - 1; q >= 0; --q) {
              run = fmaxf(run, wring[(int64_t)q * wsz + w]);
              wsuffix[(int64_t)q * wsz + w] = run;
            }
          }
        }
      }
    }
    // ---- rotate: plane t becomes the previous one, plane t + 1 the current
#pragma unroll
    for (int p = 0; p < ZPT; ++p) {
      const int l = threadIdx.x + p * TPB;
      bh0[p] = cB[0][l];
      bh1[p] = cB[1][l];
      e2pp[p] = e2p[p];
      e2p[p] = cE[2][l];
    }
    __syncthreads();
    {
      float (*te)[ZNP] = pE;
      pE = cE;
      cE = te;
      float (*tbp)[ZNP] = pB;
      pB = cB;
      cB = tbp;
    }
#pragma unroll
    for (int p = 0; p < ZPT; ++p) {
      const int l = threadIdx.x + p * TPB;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        cE[c][l] = ne[p][c];
        cB[c][l] = nb[p][c];
        ne[p][c] = ne2[p][c];
        nb[p][c] = nb2[p][c];
        jc[p][c] = jn[p][c];
      }
    }
    __syncthreads();
  }
  if (track) {
    if (__syncthreads_or(stored_nz) && threadIdx.x == 0) atomicMax(frontp, a0x + ZX - 1);
  } else {
    __syncthreads();
  }
  if (threadIdx.x == 0 && blk_hot) atomicOr(I.hot + par, 1);
  if (threadIdx.x == 0) atomicAdd(I.tiles_done + 32 * (blockIdx.x & 7), 1ull);
  if (chk != 0.0f) atomicOr(I.health, HEALTH_NONFINITE);
  if (flux_tile) {
    for (int o = 32; o > 0; o >>= 1) {
      fin += __shfl_xor(fin, o);
      fout += __shfl_xor(fout, o);
    }
    if ((threadIdx.x & 63) == 0) {
      double* ef = I.eflux + (blockIdx.x & 7) * 32;   // this XCD's line
      if (fin != 0.0) atomicAdd(ef, fin);
      if (fout != 0.0) atomicAdd(ef + 1, fout);
    }
  }
}

// Suffix maxima of the amplitude window, rebuilt after the field update of
// the step that completes a block of nwin samples (slot nwin - 1): for every
// window position w, suffix[q] = max of ring[q .. nwin - 1].  One thread per
// position, eight samples loaded at a time; a single run launches it only on
// those steps (a batch rebuilds inside the field update).
__global__ __launch_bounds__(TPB) void k_win_rebuild(const Inst I) {
  const int nwin = I.nwin;
  const int64_t wsz = I.wsz;
  const gmem<float>* __restrict__ ring = gp(I.ring);
  gmem<float>* __restrict__ suffix = gp(I.suffix);
  for (int64_t w = (int64_t)blockIdx.x * TPB + threadIdx.x; w < wsz; w += (int64_t)gridDim.x * TPB) {
    float run = 0.0f;
    int q = nwin - 1;
    for (; q >= 7; q -= 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = ring[(int64_t)(q - u) * wsz + w];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        run = fmaxf(run, v[u]);
        suffix[(int64_t)(q - u) * wsz + w] = run;
      }
    }
    for (; q >= 0; --q) {
      run = fmaxf(run, ring[(int64_t)q * wsz + w]);
      suffix[(int64_t)q * wsz + w] = run;
    }
  }
}

// ------------------------------------------------------------- ionization
template <class IT>
__device__ __forceinline__ int64_t div_ppc(const IT& I, int64_t j) {
  return I.ppc == 1 ? j : (int64_t)__umul64hi((uint64_t)j, I.ppc_magic);
}

template <int D, class IT>
__device__ __forceinline__ uint64_t neutral_id(const IT& I, int64_t jn, int& ci, int& cj, int& ck) {
  const int64_t m = div_ppc(I, jn);
  const int64_t kk = jn - m * I.ppc;
  unpack_cell(D, I.mcell[m], ci, cj, ck);
  const int64_t lin = ci + (int64_t)I.nx * (cj + (int64_t)I.ny * ck);
  return (uint64_t)(lin * I.ppc + kk);
}

// the ionization decision of one alive neutral (no side effects)
struct Birth {
  bool ev;
  int mat, ci, cj, ck;
  uint64_t id;
  float t0, t1, t2;
};
template <int D, int ORDER, class IT>
__device__ __forceinline__ Birth ionize_decide(const IT& I, int64_t jn, int ci, int cj, int ck, uint64_t id,
                                               int mat, uint32_t wx);

// Ionization of the alive neutrals with the amplitude after the field update.
// A block first marks which of its material cells can ionize at all: the
// largest windowed amplitude over the nodes any neutral of the cell can reach
// must reach the material's cut (an exact test: the shape weights are
// non-negative and sum to one).  Neutrals of the other cells read nothing more.
// A hot cell also keeps the table's bound of P up to that amplitude: each of
// its neutrals draws first, and only a draw below the bound (a few times the
// step's events) loads the neutral and gathers its amplitude.  The decision
// is the same as gathering first: the gathered amplitude never exceeds the
// cell's largest (times 1 + 2^-16, which covers the FP32 sum of non-negative
// weights), and the bound covers the lookup at every amplitude below it.
template <int D, int ORDER, class IT>
__device__ __forceinline__ void ionize_births(const IT& I, const Birth& b, int64_t jn, int step);

template <int D, int ORDER, bool ONE>
__global__ __launch_bounds__(TPB, 8) void k_ionize(Group g, std::conditional_t<ONE, Inst, NoInst> one) {
  __shared__ unsigned char hot[TPB + 2];
  __shared__ float spb[TPB + 2];        // bound of P over the cell's reachable amplitudes
  __shared__ TabSeg sseg[ION_SMAT][ION_SSEG];   // rate-table segments (while they fit)
  __shared__ int snseg[ION_SMAT];
  __shared__ float sasat[ION_SMAT];
  __shared__ uint32_t scell[TPB + 2];   // packed cell and material of each cell of the block
  __shared__ signed char smat[TPB + 2];
  const Slot sl = ONE ? Slot{0, (int)blockIdx.x, g.blocks} : block_slot(g);
  auto& I = inst_of(g, sl.ii, one);
  const int step = ONE || g.step >= 0 ? g.step : I.step_now;
  // the flag of the next step is raised by its field update, which runs after
  // this kernel; a cold grid (no amplitude at any cut) ionizes nothing
  if (sl.bk == 0 && threadIdx.x == 0) I.hot[(step + 1) & 1] = 0;
  if (!I.hot[step & 1]) return;
  // a block takes TPB x nit consecutive neutrals, nit = min(ppc, ION_NIT):
  // at most TPB cells, whose per-cell pass then keeps every thread busy
  const int nit = ion_nit(I.ppc);
  const int64_t span = (int64_t)TPB * nit;
  const int64_t j0 = (int64_t)xcd_remap(sl.bk, sl.nbk) * span;
  const int64_t nneut = I.nneut;
  if (j0 >= nneut) return;
  const int64_t m0 = div_ppc(I, j0);
  const int64_t jl = (j0 + span < nneut ? j0 + span : nneut) - 1;
  const int ncell = (int)(div_ppc(I, jl) - m0 + 1);
  // the rate tables' segments, staged while the cells' amplitudes load
  for (int e = threadIdx.x; e < ION_SMAT * ION_SSEG; e += TPB) {
    const int m = e / ION_SSEG, q = e % ION_SSEG;
    if (m < I.nmat) {
      const TabHdr* h = I.tab[m];
      const int ns = h->nseg;
      if (q == 0) {
        snseg[m] = ns;
        sasat[m] = h->asat;
      }
      if (q < ns && ns <= ION_SSEG) sseg[m][q] = reinterpret_cast<const TabSeg*>(h + 1)[q];
    }
  }
  for (int t = threadIdx.x; t < ncell; t += TPB) {
    int ci, cj, ck;
    const uint32_t pc = I.mcell[m0 + t];
    unpack_cell(D, pc, ci, cj, ck);
    const int mat = I.mat_cell[ci];
    scell[t] = pc;
    smat[t] = (signed char)mat;
    constexpr int lo = ORDER == 2 ? -1 : 0, hi = ORDER == 2 ? 2 : 1;
    float amax = 0.0f;
    for (int c = (D >= 3 ? lo : 0); c <= (D >= 3 ? hi : 0); ++c) {
      const int oz = D >= 3 ? I.sz * (wrapi(ck + c, I.nz, I.per_z) + I.Gz) : 0;
      for (int b = (D >= 2 ? lo : 0); b <= (D >= 2 ? hi : 0); ++b) {
        const int oy = D >= 2 ? I.sy * (wrapi(cj + b, I.ny, I.per_y) + I.Gy) : 0;
        for (int a = lo; a <= hi; ++a) amax = fmaxf(amax, I.A[ci + a + G + oy + oz]);
      }
    }
    // a cell whose neutrals have all been ionized needs no per-neutral pass
    const int64_t a0 = (m0 + t) * I.ppc, a1 = a0 + I.ppc;
    bool alive = false;
    for (int64_t w = a0 >> 5; w <= ((a1 - 1) >> 5) && !alive; ++w) {
      const int lo_b = (int)((a0 > 32 * w ? a0 : 32 * w) - 32 * w);
      const int hi_b = (int)((a1 < 32 * w + 32 ? a1 : 32 * w + 32) - 32 * w);
      const uint32_t mask = hi_b - lo_b == 32 ? ~0u : ((1u << (hi_b - lo_b)) - 1u) << lo_b;
      alive = (I.alive[w] & mask) != 0u;
    }
    const bool h = alive && mat >= 0 && amax >= I.acut[mat];
    hot[t] = h;
    spb[t] = h ? amax * (1.0f + 0x1p-16f) : 0.0f;   // the bound's amplitude, bound below
  }
  __syncthreads();
  for (int t = threadIdx.x; t < ncell; t += TPB) {
    if (!hot[t]) continue;
    const int mat = smat[t];
    const TabHdr* h = I.tab[mat];
    const bool st = mat < ION_SMAT && snseg[mat] <= ION_SSEG;
    spb[t] = st ? table_bound_at(h, I.acut[mat], sasat[mat], snseg[mat], sseg[mat], spb[t]) : table_bound(h, spb[t]);
  }
  __syncthreads();
  for (int it = 0; it < nit; ++it) {
    const int64_t jn = j0 + (int64_t)it * TPB + threadIdx.x;
    Birth b{};
    if (jn < nneut) {
      const int64_t mn = div_ppc(I, jn);
      const int t = (int)(mn - m0);
      if (hot[t]) {
        int ci, cj, ck;
        unpack_cell(D, scell[t], ci, cj, ck);
        const int64_t lin = ci + (int64_t)I.nx * (cj + (int64_t)I.ny * ck);
        const uint64_t id = (uint64_t)(lin * I.ppc + (jn - mn * I.ppc));
        const u32x4 w = draw(I.seed, id, (uint32_t)(step + 1), PURPOSE_IONIZE);
        if ((double)w.x + 0.5 < (double)spb[t] * 4294967296.0)
          b = ionize_decide<D, ORDER>(I, jn, ci, cj, ck, id, smat[t], w.x);
      }
    }
    ionize_births<D, ORDER>(I, b, jn, step);
  }
}

// The events of one wave (64 consecutive neutrals starting at a multiple of
// 64): one slot reservation per tile, one event count per material, one
// alive-mask update per 32-neutral word, then each event's two carriers.
template <int D, int ORDER, class IT>
__device__ __forceinline__ void ionize_births(const IT& I, const Birth& b, int64_t jn, int step) {
  const unsigned long long m = __ballot(b.ev);
  if (!m) return;
  const int lane = threadIdx.x & 63;
  // birth slots: the tile's birth room (electron and positive-carrier halves)
  // while it lasts, else two slots after the layout
  int tt = -1;
  if (b.ev) {
    const int t = tile_of<D>(I, pack_cell(D, b.ci, b.cj, b.ck));
    tt = t >= 0 && I.tslack[t] > 0 ? t : -1;
  }
  const int r = wave_rank_add(I.tfill, tt);
  int cap = 0;
  if (tt >= 0) cap = I.tslack[tt];
  const bool room = tt >= 0 && r < cap;
  int se = 0, sp = 0;
  if (room) {
    se = I.tbirth[tt] + r;
    sp = se + cap;
  }
  const unsigned long long mt = __ballot(b.ev && !room);
  if (mt) {
    const int leader = __ffsll((long long)mt) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(I.pcount, 2 * __popcll(mt));
    base = __shfl(base, leader);
    se = base + 2 * __popcll(mt & ((1ull << lane) - 1ull));
    sp = se + 1;
  }
  if (lane == 0 && (unsigned)m) atomicAnd(&I.alive[jn >> 5], ~(unsigned)m);
  if (lane == 32 && (unsigned)(m >> 32)) atomicAnd(&I.alive[jn >> 5], ~(unsigned)(m >> 32));
  for (unsigned long long left = m; left;) {
    const int l0 = __ffsll((long long)left) - 1;
    const int mt = __shfl(b.mat, l0);
    const unsigned long long same = __ballot(b.ev && b.mat == mt);
    if (lane == l0) atomicAdd(&I.nevents[(blockIdx.x & 7) * 32 + mt], (unsigned long long)__popcll(same));
    left &= ~same;
  }
  if (!b.ev) return;
  const int n1 = step + 1;
  I.death[jn] = n1;
  if (!room && se + 2 > I.capacity) {
    atomicOr(I.health, HEALTH_CAPACITY);
    return;
  }
  float ux, uy, uz;
  maxwell(I.seed, b.id, PURPOSE_VEL, I.ksig[b.mat], ux, uy, uz);
  const uint32_t pc = pack_cell(D, b.ci, b.cj, b.ck);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int q = s == 0 ? se : sp;
    I.pcell[q] = pc;
    I.po0[q] = off_fix(b.t0);
    if (D >= 2) I.po1[q] = off_fix(b.t1);
    if (D >= 3) I.po2[q] = off_fix(b.t2);
    I.pu0[q] = ux;
    I.pu1[q] = uy;
    I.pu2[q] = uz;
    I.pkind[q] = (uint8_t)(2 * b.mat + s);
    I.pid[q] = (uint32_t)b.id;
  }
}

__global__ void k_advance(Inst* insts, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const int s = *insts[i].step + 1;
    *insts[i].step = s;
    insts[i].step_now = s;
  }
}

// A neutral whose draw fell below its cell's bound: the alive bit and the
// offsets (loaded together, one round trip), the amplitude gathered at the
// neutral, the exact FP64 comparison of the draw with P.
template <int D, int ORDER, class IT>
__device__ __forceinline__ Birth ionize_decide(const IT& I, int64_t jn, int ci, int cj, int ck, uint64_t id,
                                               int mat, uint32_t wx) {
  Birth b{};
  const uint32_t aw = I.alive[jn >> 5];
  b.t0 = I.no0[jn];
  b.t1 = D >= 2 ? I.no1[jn] : 0.f;
  b.t2 = D >= 3 ? I.no2[jn] : 0.f;
  if (!((aw >> (jn & 31)) & 1u)) return b;
  b.ci = ci;
  b.cj = cj;
  b.ck = ck;
  b.id = id;
  // amplitude at the neutral: node-shape gather of A
  Axis<ORDER> X, Y, Z;
  make_axis<ORDER>(X, ci, b.t0, I.nx, 0, G, 1);
  if (D >= 2) make_axis<ORDER>(Y, cj, b.t1, I.ny, I.per_y, I.Gy, I.sy);
  if (D >= 3) make_axis<ORDER>(Z, ck, b.t2, I.nz, I.per_z, I.Gz, I.sz);
  const float Ap = gather<D, ORDER>(I.A, X, Y, Z, 0, 0, 0);
  b.mat = mat;
  if (mat < 0 || !(Ap >= I.acut[mat])) return b;
  const float P = table_lookup(I.tab[mat], Ap);
  // event iff (w + 1/2) 2^-32 < P, decided exactly in FP64
  b.ev = (double)wx + 0.5 < (double)P * 4294967296.0;
  return b;
}

// ------------------------------------------------------------------ setup
template <int D>
__global__ __launch_bounds__(TPB) void k_init_neutrals(const Inst* d) {
  const Inst& I = *d;
  const int64_t jn = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (jn >= I.nneut) return;
  int ci, cj, ck;
  const uint64_t id = neutral_id<D>(I, jn, ci, cj, ck);
  const u32x4 w = draw(I.seed, id, 0u, PURPOSE_POS);
  // offsets (w >> 8) 2^-24: FP32 numbers in [0, 1)
  I.no0[jn] = (float)(w.x >> 8) * 0x1p-24f;
  if (D >= 2) I.no1[jn] = (float)(w.y >> 8) * 0x1p-24f;
  if (D >= 3) I.no2[jn] = (float)(w.z >> 8) * 0x1p-24f;
  I.death[jn] = -1;
  if ((jn & 31) == 0) {
    const int64_t left = I.nneut - jn;
    I.alive[jn >> 5] = left >= 32 ? 0xFFFFFFFFu : ((1u << left) - 1u);
  }
}

template <int D>
__global__ __launch_bounds__(TPB) void k_preionize(const Inst* d, const float* sig_e, const float* sig_p) {
  const Inst& I = *d;
  const int64_t jn = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (jn >= I.nneut) return;
  int ci, cj, ck;
  const uint64_t id = neutral_id<D>(I, jn, ci, cj, ck);
  const int mat = I.mat_cell[ci];
  I.death[jn] = 0;
  if ((jn & 31) == 0) I.alive[jn >> 5] = 0u;
  const uint32_t pc = pack_cell(D, ci, cj, ck);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    float ux, uy, uz;
    maxwell(I.seed, id, s == 0 ? PURPOSE_STRESS_E : PURPOSE_STRESS_P, s == 0 ? sig_e[mat] : sig_p[mat],
            ux, uy, uz);
    // every neutral's pair sits in slots 2j, 2j + 1 (cell order kept)
    const int64_t q = 2 * jn + s;
    I.pcell[q] = pc;
    I.po0[q] = off_fix(I.no0[jn]);
    if (D >= 2) I.po1[q] = off_fix(I.no1[jn]);
    if (D >= 3) I.po2[q] = off_fix(I.no2[jn]);
    I.pu0[q] = ux;
    I.pu1[q] = uy;
    I.pu2[q] = uz;
    I.pkind[q] = (uint8_t)(2 * mat + s);
    I.pid[q] = (uint32_t)id;
  }
}

// ------------------------------------------------------------ diagnostics
// acc layout: [kind][0] count, [kind][1] sum weight * KE (J)
__global__ __launch_bounds__(TPB) void k_diag_particles(const Inst* d, double* acc) {
  const Inst& I = *d;
  __shared__ double sh[MAXKIND * 2];
  for (int q = threadIdx.x; q < MAXKIND * 2; q += TPB) sh[q] = 0.0;
  __syncthreads();
  int count = *I.pcount;
  count = count < I.capacity ? count : I.capacity;
  for (int p = blockIdx.x * TPB + threadIdx.x; p < count; p += gridDim.x * TPB) {
    const uint8_t kd = I.pkind[p];
    if (kd == DEAD) continue;
    const double ux = I.pu0[p], uy = I.pu1[p], uz = I.pu2[p];
    const double u2 = ux * ux + uy * uy + uz * uz;
    const double c = 299792458.0;
    const double ke = I.kmass[kd] * c * c * u2 / (sqrt(1.0 + u2) + 1.0) * I.kw[kd];
    atomicAdd(&sh[2 * kd], 1.0);
    atomicAdd(&sh[2 * kd + 1], ke);
  }
  __syncthreads();
  for (int q = threadIdx.x; q < MAXKIND * 2; q += TPB)
    if (sh[q] != 0.0) atomicAdd(&acc[q], sh[q]);
}

// Energy histogram (Sec. 5: the electrons' energy distribution in one layer,
// fitted with a chi^2 law).  Kinetic energy m c^2 |u|^2 / (gamma + 1) in FP64,
// every operation rounded on its own in the order written (no contraction), so
// the bin a particle falls in is the one the same formula gives anywhere; the
// bin is found by bisection over the caller's edges (staged in LDS): column 0
// below the first edge, column j in [edge j-1, edge j), the last column at or
// above the last.  Counts per kind in LDS (when they fit) or straight to HBM.
// One 1024-thread block per CU at most: each block adds its counts to HBM
// once, so a column takes at most one atomic per CU.
constexpr int SPEC_TPB = 1024;
template <int D>
__global__ __launch_bounds__(SPEC_TPB) void k_spectrum(const Inst* d, SpecArgs a, const double* edges,
                                                       unsigned long long* out) {
  extern __shared__ double se[];   // nedges edges, then (a.lds) the counts
  unsigned int* sc = (unsigned int*)(se + a.nedges);
  const Inst& I = *d;
  const int ncol = a.nedges + 1, ncnt = a.nkinds * ncol;
  for (int q = threadIdx.x; q < a.nedges; q += SPEC_TPB) se[q] = edges[q];
  if (a.lds)
    for (int q = threadIdx.x; q < ncnt; q += SPEC_TPB) sc[q] = 0u;
  __syncthreads();
  int count = *I.pcount;
  count = count < I.capacity ? count : I.capacity;
  for (int p = blockIdx.x * SPEC_TPB + threadIdx.x; p < count; p += gridDim.x * SPEC_TPB) {
    const int kd = I.pkind[p];
    if (kd == DEAD || kd >= a.nkinds) continue;
    if (a.x_hi > a.x_lo) {
      int ci, cj, ck;
      unpack_cell(D, I.pcell[p], ci, cj, ck);
      if (ci < a.x_lo || ci >= a.x_hi) continue;
    }
    double ke;
    {
#pragma clang fp contract(off)
      const double ux = I.pu0[p], uy = I.pu1[p], uz = I.pu2[p];
      const double u2 = ux * ux + uy * uy + uz * uz;
      ke = a.mc2_eV[kd] * u2 / (sqrt(1.0 + u2) + 1.0);
    }
    // number of edges at or below ke
    int lo = 0, hi = a.nedges;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (se[mid] <= ke) lo = mid + 1; else hi = mid;
    }
    const int q = kd * ncol + lo;
    if (a.lds) atomicAdd(&sc[q], 1u);
    else atomicAdd(&out[q], 1ull);
  }
  if (a.lds) {
    __syncthreads();
    for (int q = threadIdx.x; q < ncnt; q += SPEC_TPB)
      if (sc[q]) atomicAdd(&out[q], (unsigned long long)sc[q]);
  }
}

// Trajectory sampling (Sec. 5: tracks of a random 2 % of the electrons): a
// live particle is sampled iff the first word of the Philox block
// (seed; id, 0, TRACK) is below thr, so an electron and its positive carrier
// (one id) go together and the choice does not depend on the slot.  A block
// takes chunks of TRACK_CHUNK slots: the sampled slots of a chunk are listed
// in LDS (one LDS atomic per wave), the chunk reserves its records with one
// HBM atomic, then writes them.  Records beyond max_records are counted but
// not written.
constexpr int TRACK_CHUNK = 4096, TRACK_TPB = 1024;
template <int D>
__global__ __launch_bounds__(TRACK_TPB) void k_tracks(const Inst* d, uint32_t thr, int step, TrackRec* rec,
                                                unsigned long long* n, int64_t max_records) {
  __shared__ unsigned slist[TRACK_CHUNK];
  __shared__ unsigned scount;
  __shared__ unsigned long long sbase;
  const Inst& I = *d;
  int count = *I.pcount;
  count = count < I.capacity ? count : I.capacity;
  const int lane = threadIdx.x & 63;
  for (int c0 = blockIdx.x * TRACK_CHUNK; c0 < count; c0 += gridDim.x * TRACK_CHUNK) {
    if (threadIdx.x == 0) scount = 0u;
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < TRACK_CHUNK / TRACK_TPB; ++k) {
      const int p = c0 + k * TRACK_TPB + threadIdx.x;
      bool sel = false;
      if (p < count && I.pkind[p] != DEAD) sel = draw(I.seed, (uint64_t)I.pid[p], 0u, PURPOSE_TRACK).x < thr;
      const unsigned long long m = __ballot(sel);
      if (m) {
        const int leader = __ffsll((long long)m) - 1;
        unsigned wb = 0u;
        if (lane == leader) wb = atomicAdd(&scount, (unsigned)__popcll(m));
        wb = (unsigned)__shfl((int)wb, leader);
        if (sel) slist[wb + (unsigned)__popcll(m & ((1ull << lane) - 1ull))] = (unsigned)p;
      }
    }
    __syncthreads();
    const unsigned cnt = scount;
    if (threadIdx.x == 0) sbase = cnt ? atomicAdd(n, (unsigned long long)cnt) : 0ull;
    __syncthreads();
    const unsigned long long base = sbase;
    for (unsigned i = threadIdx.x; i < cnt; i += TRACK_TPB) {
      if ((int64_t)(base + i) >= max_records) break;
      const int p = (int)slist[i];
      int ci, cj, ck;
      unpack_cell(D, I.pcell[p], ci, cj, ck);
      TrackRec r;
      r.id = I.pid[p];
      r.kind = I.pkind[p];
      r.step = step;
      r.cell[0] = ci;
      r.cell[1] = cj;
      r.cell[2] = ck;
      r.off[0] = off_f32(I.po0[p]);
      r.off[1] = D >= 2 ? off_f32(I.po1[p]) : 0.0f;
      r.off[2] = D >= 3 ? off_f32(I.po2[p]) : 0.0f;
      r.pad = 0;
      rec[base + i] = r;
    }
    __syncthreads();
  }
}

// Maximum accumulated intensity (Sec. 5, multilayer mirror): each domain
// node's |E|^2, the Yee components averaged to the node (positions outside the
// box count as zero, periodic axes wrap), raises the node's running maximum.
// One thread per domain node, x fastest.
__global__ __launch_bounds__(TPB) void k_imax(ImaxArgs a, float* __restrict__ imax) {
  const int64_t n = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (n >= a.nodes) return;
  const int i = (int)(n % a.mx);
  const int j = (int)((n / a.mx) % a.my);
  const int k = (int)(n / ((int64_t)a.mx * a.my));
  const int64_t o = (int64_t)(i + G) + (int64_t)a.sy * (j + a.Gy) + (int64_t)a.sz * (k + a.Gz);
  // component c at node (i, j, k): mean of its two half-integer neighbours
  // along axis c when c is a present axis, else its value at the node
  auto node = [&](const float* F, int c) -> float {
    if (c >= a.D) return F[o];
    const int v = c == 0 ? i : c == 1 ? j : k;
    const int nv = c == 0 ? a.nx : c == 1 ? a.ny : a.nz;
    const bool per = c == 1 ? a.per_y : c == 2 ? a.per_z : false;
    const int64_t st = c == 0 ? 1 : c == 1 ? a.sy : a.sz;
    const float hiv = v < nv ? F[o] : 0.0f;
    float lov;
    if (v >= 1) lov = F[o - st];
    else lov = per ? F[o + (int64_t)(nv - 1) * st] : 0.0f;
    return 0.5f * (lov + hiv);
  };
  const float ex = node(a.E0, 0), ey = node(a.E1, 1), ez = node(a.E2, 2);
  const float v = ex * ex + ey * ey + ez * ez;
  if (v > imax[o]) imax[o] = v;
}

__global__ __launch_bounds__(TPB) void k_diag_field_energy(const Inst* d, int64_t ncell, double* acc) {
  const Inst& I = *d;
  const int par = *I.step & 1;
  double s = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * TPB + threadIdx.x; p < ncell; p += (int64_t)gridDim.x * TPB) {
    const int ai = (int)(p % I.Px);
    const double ex = I.F[par][0][p], ey = I.F[par][1][p], ez = I.F[par][2][p];
    s += ex * ex / I.ie_half[ai] + (ey * ey + ez * ez) / I.ie_node[ai];
    const double bx = I.F[par][3][p], by = I.F[par][4][p], bz = I.F[par][5][p];
    s += bx * bx + by * by + bz * bz;
  }
  __shared__ double sh[TPB];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = TPB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(acc, sh[0]);
}

// what: 0 = rho/eps0 (all charged), 1 = electron number density, 2 = electron
// energy density; FP64 node grid in the padded layout
template <int D, int ORDER>
__global__ __launch_bounds__(TPB) void k_diag_deposit(const Inst* d, double* grid, int what) {
  const Inst& I = *d;
  int count = *I.pcount;
  count = count < I.capacity ? count : I.capacity;
  for (int p = blockIdx.x * TPB + threadIdx.x; p < count; p += gridDim.x * TPB) {
    const uint8_t kd = I.pkind[p];
    if (kd == DEAD) continue;
    if (what > 0 && (kd & 1)) continue;
    double val;
    if (what == 0) {
      val = I.kqhat[kd];
    } else if (what == 1) {
      val = I.kw[kd] / I.vcell;
    } else {
      const double ux = I.pu0[p], uy = I.pu1[p], uz = I.pu2[p];
      const double u2 = ux * ux + uy * uy + uz * uz;
      const double c = 299792458.0;
      val = I.kw[kd] * I.kmass[kd] * c * c * u2 / (sqrt(1.0 + u2) + 1.0) / I.vcell;
    }
    int ci, cj, ck;
    unpack_cell(D, I.pcell[p], ci, cj, ck);
    Axis<ORDER> X, Y, Z;
    make_axis<ORDER>(X, ci, off_f32(I.po0[p]), I.nx, 0, G, 1);
    if (D >= 2) make_axis<ORDER>(Y, cj, off_f32(I.po1[p]), I.ny, I.per_y, I.Gy, I.sy);
    if (D >= 3) make_axis<ORDER>(Z, ck, off_f32(I.po2[p]), I.nz, I.per_z, I.Gz, I.sz);
    constexpr int SY = D >= 2 ? ORDER + 1 : 1;
    constexpr int SZ = D >= 3 ? ORDER + 1 : 1;
    for (int c = 0; c < SZ; ++c)
      for (int b = 0; b < SY; ++b)
        for (int a = 0; a <= ORDER; ++a) {
          const double w = (double)X.wn[a] * (D >= 2 ? (double)Y.wn[b] : 1.0) * (D >= 3 ? (double)Z.wn[c] : 1.0);
          atomicAdd(&grid[X.on[a] + (D >= 2 ? Y.on[b] : 0) + (D >= 3 ? Z.on[c] : 0)], val * w);
        }
  }
}

// Gauss residual div(E/ie) - rho/eps0 at interior nodes: acc[0] = max |res|
// (as uint64 bits of a non-negative double), acc[1] = max |rho/eps0|
template <int D>
__global__ __launch_bounds__(TPB) void k_diag_gauss(const Inst* d, const double* rho, double* acc) {
  const Inst& I = *d;
  const int64_t ncell = (int64_t)I.Px * I.Py * I.Pz;
  const int par = *I.step & 1;
  const float* E0 = I.F[par][0];
  const float* E1 = I.F[par][1];
  const float* E2 = I.F[par][2];
  // displacement E / ie + Q + chi3 E^3 (Q = P / eps0 of Lorentz media, chi3
  // the Kerr term; ai the padded x index of the position)
  const bool lor = I.lx0 < I.lx1;
  auto dsp = [&](int c, const float* E, int64_t q, float ie, int ai) {
    const double e = E[q];
    if (!lor) return e / ie;
    const double chi = c == 0 ? I.lor_half[ai].w : I.lor_node[ai].w;
    return e / ie + (double)I.Q[par][c][q] + chi * e * e * e;
  };
  double mres = 0.0, mrho = 0.0, sres = 0.0, nres = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * TPB + threadIdx.x; p < ncell; p += (int64_t)gridDim.x * TPB) {
    int i, j, k;
    decode<D>(I, p, i, j, k);
    if (i < 1 || i > I.nx - 1) continue;
    if (D >= 2 && (I.per_y ? (j < 0 || j >= I.ny) : (j < 1 || j > I.ny - 1))) continue;
    if (D >= 3 && (I.per_z ? (k < 0 || k >= I.nz) : (k < 1 || k > I.nz - 1))) continue;
    const int ai = i + G;
    double div = (dsp(0, E0, p, I.ie_half[ai], ai) - dsp(0, E0, p - 1, I.ie_half[ai - 1], ai - 1)) / I.dx[0];
    if (D >= 2) {
      const int dym = I.per_y && j == 0 ? (I.ny - 1) * I.sy : -I.sy;
      div += (dsp(1, E1, p, I.ie_node[ai], ai) - dsp(1, E1, p + dym, I.ie_node[ai], ai)) / I.dx[1];
    }
    if (D >= 3) {
      const int dzm = I.per_z && k == 0 ? (I.nz - 1) * I.sz : -I.sz;
      div += (dsp(2, E2, p, I.ie_node[ai], ai) - dsp(2, E2, p + dzm, I.ie_node[ai], ai)) / I.dx[2];
    }
    const double r = div - rho[p];
    mres = fmax(mres, fabs(r));
    mrho = fmax(mrho, fabs(rho[p]));
    sres += r * r;
    nres += 1.0;
  }
  atomicMax(reinterpret_cast<unsigned long long*>(acc), __double_as_longlong(mres));
  atomicMax(reinterpret_cast<unsigned long long*>(acc) + 1, __double_as_longlong(mrho));
  // sum of squares and count of the interior nodes (root mean square on the host)
  if (nres > 0.0) {
    atomicAdd(acc + 2, sres);
    atomicAdd(acc + 3, nres);
  }
}

__global__ void k_table_probe(const TabHdr* tab, const float* A, float* P, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) P[i] = table_lookup(tab, A[i]);
}

// ------------------------------------------------------------- launchers
#define DISPATCH_D(D, ...)                                    \
  switch (D) {                                                \
    case 1: { constexpr int DD = 1; __VA_ARGS__; break; }     \
    case 2: { constexpr int DD = 2; __VA_ARGS__; break; }     \
    default: { constexpr int DD = 3; __VA_ARGS__; break; }    \
  }

// plain launch, or one that stamps the events it is given
#define GO(K, grid, block, s, e0, e1, ...)                                               \
  do {                                                                                    \
    if ((e0) || (e1))                                                                     \
      hipExtLaunchKernelGGL(K, dim3(grid), dim3(block), 0, s, e0, e1, 0, __VA_ARGS__);    \
    else                                                                                  \
      hipLaunchKernelGGL(K, dim3(grid), dim3(block), 0, s, __VA_ARGS__);                  \
  } while (0)

// a single run passes its parameter block by value (see k_fields)
#define ONE_OR_GROUP(KT, tpb, ...)                                                    \
  do {                                                                                \
    if (one)                                                                          \
      GO((KT<__VA_ARGS__, true>), g.blocks, tpb, s, st.start, st.stop, g, *g.host);   \
    else                                                                              \
      GO((KT<__VA_ARGS__, false>), g.blocks, tpb, s, st.start, st.stop, g, NoInst{}); \
  } while (0)
int push_grid(int D) {
  int dev = 0, bpc = 0;
  hipDeviceProp_t pr{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&pr, dev) != hipSuccess) return 0;
  hipError_t e = hipSuccess;
  switch (D) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, k_push<1, 2, false, false, true>, push_tpb(1), 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, k_push<2, 2, true, false, true>, push_tpb(2), 0); break;
    default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, k_push<3, 2, true, true, true>, push_tpb(3), 0); break;
  }
  if (e != hipSuccess || bpc < 1) return 0;
  return std::max(8, bpc * pr.multiProcessorCount / 8 * 8);
}
void launch_push(const Group& g, int D, int order, bool per, hipStream_t s, Stamp st) {
  const bool one = g.n == 1 && g.host && g.step >= 0;
  // periodic transverse axes are a template parameter (D >= 2)
  if (order == 1) {
    if (per && D >= 2) {
      DISPATCH_D(D, ONE_OR_GROUP(k_push, push_tpb(DD), DD, 1, DD >= 2, DD >= 3));
    } else {
      DISPATCH_D(D, ONE_OR_GROUP(k_push, push_tpb(DD), DD, 1, false, false));
    }
  } else {
    if (per && D >= 2) {
      DISPATCH_D(D, ONE_OR_GROUP(k_push, push_tpb(DD), DD, 2, DD >= 2, DD >= 3));
    } else {
      DISPATCH_D(D, ONE_OR_GROUP(k_push, push_tpb(DD), DD, 2, false, false));
    }
  }
}
void launch_sort(const Group& gp, const Group& gscan, int D, hipStream_t s, Stamp st) {
  hipEvent_t none = nullptr;
  DISPATCH_D(D, GO((k_sort_count<DD>), gp.blocks, TPB, s, st.start, none, gp));
  DISPATCH_D(D, GO((k_sort_scan<DD>), gscan.blocks, SCAN_TPB, s, none, none, gscan));
  DISPATCH_D(D, GO((k_sort_fill<DD>), gp.blocks, TPB, s, none, none, gp));
  DISPATCH_D(D, GO((k_sort_scatter<DD>), gp.blocks, TPB, s, none, none, gp));
  DISPATCH_D(D, GO((k_sort_copy<DD>), gp.blocks, TPB, s, none, st.stop, gp));
}
#define FIELDS_V(DD, V)                                \
  do {                                                 \
    if (g.lor == 2)                                    \
      ONE_OR_GROUP(k_fields, TPB, DD, V, 2);           \
    else if (g.lor)                                    \
      ONE_OR_GROUP(k_fields, TPB, DD, V, 1);           \
    else                                               \
      ONE_OR_GROUP(k_fields, TPB, DD, V, 0);           \
  } while (0)
void launch_fields(const Group& g, int D, int variant, hipStream_t s, Stamp st) {
  const bool one = g.n == 1 && g.host && g.front && g.xext && g.step >= 0;
  switch (variant) {
    case 1: DISPATCH_D(D, FIELDS_V(DD, 1)); break;
    case 2: DISPATCH_D(D, FIELDS_V(DD, 2)); break;
    case 3: DISPATCH_D(D, FIELDS_V(DD, 3)); break;
    case 4: DISPATCH_D(D, FIELDS_V(DD, 4)); break;
    case 5: DISPATCH_D(D, FIELDS_V(DD, 5)); break;
    case 6: DISPATCH_D(D, FIELDS_V(DD, 6)); break;
    case kMarchVariant:
      if (D == 3) {
        if (one && g.lor == 2)
          GO((k_fields_z<true, 2>), g.blocks, TPB, s, st.start, st.stop, g, *g.host);
        else if (one && g.lor)
          GO((k_fields_z<true, 1>), g.blocks, TPB, s, st.start, st.stop, g, *g.host);
        else if (one)
          GO((k_fields_z<true, 0>), g.blocks, TPB, s, st.start, st.stop, g, *g.host);
        else if (g.lor == 2)
          GO((k_fields_z<false, 2>), g.blocks, TPB, s, st.start, st.stop, g, NoInst{});
        else if (g.lor)
          GO((k_fields_z<false, 1>), g.blocks, TPB, s, st.start, st.stop, g, NoInst{});
        else
          GO((k_fields_z<false, 0>), g.blocks, TPB, s, st.start, st.stop, g, NoInst{});
        break;
      }
      [[fallthrough]];
    default: DISPATCH_D(D, FIELDS_V(DD, 0)); break;
  }
}
int field_tiles(int D, int variant, int Px, int Py, int Pz) {
  const TileShape t = tile_shape(D, variant);
  if (D == 3 && variant == kMarchVariant) {
    // x over the padded array, y and z over the box (padded extents are
    // n + 1 + 2 G); z cut into as many segments as fill the resident blocks
    const int ny = Py - 1 - 2 * G, nz = Pz - 1 - 2 * G;
    const int cols = ((Px + t.x - 1) / t.x) * ((ny + t.y - 1) / t.y);
    static int slots = 0;
    if (!slots) {
      int dev = 0, bpc = 0;
      hipDeviceProp_t pr{};
      if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&pr, dev) == hipSuccess &&
          hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, k_fields_z<true, 0>, TPB, 0) == hipSuccess && bpc > 0)
        slots = bpc * pr.multiProcessorCount;
      else
        slots = 1024;
    }
    const int want = std::max(1, std::min(nz, slots / std::max(1, cols)));
    const int zs = (nz + want - 1) / want;
    return cols * ((nz + zs - 1) / zs);
  }
  return ((Px + t.x - 1) / t.x) * (D >= 2 ? (Py + t.y - 1) / t.y : 1) * (D >= 3 ? (Pz + t.z - 1) / t.z : 1);
}
int field_tile_variants(int D, bool periodic_yz) { return D == 3 && periodic_yz ? kTileVariants : kTileVariants - 1; }
int field_tile_x(int D, int variant) { return tile_shape(D, variant).x; }
void launch_win_rebuild(const Inst& I, int64_t wsz, hipStream_t s, hipEvent_t stop) {
  if (wsz <= 0) return;
  const int64_t nb = std::min<int64_t>((wsz + TPB - 1) / TPB, 4096);
  hipEvent_t none = nullptr;
  GO(k_win_rebuild, (unsigned)nb, TPB, s, none, stop, I);
}
void launch_ionize(const Group& g, int D, int order, hipStream_t s, Stamp st) {
  const bool one = g.n == 1 && g.host && g.step >= 0;
  if (order == 1) {
    DISPATCH_D(D, ONE_OR_GROUP(k_ionize, TPB, DD, 1));
  } else {
    DISPATCH_D(D, ONE_OR_GROUP(k_ionize, TPB, DD, 2));
  }
}
void launch_advance(Inst* insts, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3((n + 63) / 64), dim3(64), 0, s, insts, n);
}
void launch_init_neutrals_d(const Inst* d, int64_t nneut, int D, hipStream_t s) {
  if (nneut <= 0) return;
  const unsigned nb = (unsigned)((nneut + TPB - 1) / TPB);
  DISPATCH_D(D, hipLaunchKernelGGL((k_init_neutrals<DD>), dim3(nb), dim3(TPB), 0, s, d));
}
void launch_preionize_d(const Inst* d, int64_t nneut, int D, const float* se, const float* sp,
                        hipStream_t s) {
  if (nneut <= 0) return;
  const unsigned nb = (unsigned)((nneut + TPB - 1) / TPB);
  DISPATCH_D(D, hipLaunchKernelGGL((k_preionize<DD>), dim3(nb), dim3(TPB), 0, s, d, se, sp));
}
void launch_diag_particles(const Inst* d, int capacity, double* acc, hipStream_t s) {
  unsigned nb = (unsigned)((capacity + TPB - 1) / TPB);
  nb = nb < 1 ? 1 : (nb > 2048 ? 2048 : nb);
  hipLaunchKernelGGL(k_diag_particles, dim3(nb), dim3(TPB), 0, s, d, acc);
}
void launch_spectrum(const Inst* d, int D, int capacity, const SpecArgs& a, const double* edges,
                     unsigned long long* out, hipStream_t s) {
  unsigned nb = (unsigned)((capacity + SPEC_TPB - 1) / SPEC_TPB);
  nb = nb < 1 ? 1 : (nb > 256 ? 256 : nb);
  const size_t lds = sizeof(double) * a.nedges + (a.lds ? sizeof(unsigned) * a.nkinds * (a.nedges + 1) : 0);
  DISPATCH_D(D, hipLaunchKernelGGL((k_spectrum<DD>), dim3(nb), dim3(SPEC_TPB), lds, s, d, a, edges, out));
}
void launch_tracks(const Inst* d, int D, int capacity, uint32_t thr, int step, TrackRec* rec,
                   unsigned long long* n, int64_t max_records, hipStream_t s) {
  unsigned nb = (unsigned)((capacity + TRACK_CHUNK - 1) / TRACK_CHUNK);
  nb = nb < 1 ? 1 : (nb > 1024 ? 1024 : nb);
  DISPATCH_D(D, hipLaunchKernelGGL((k_tracks<DD>), dim3(nb), dim3(TRACK_TPB), 0, s, d, thr, step, rec, n, max_records));
}
void launch_imax(const ImaxArgs& a, float* imax, hipStream_t s) {
  if (a.nodes <= 0) return;
  hipLaunchKernelGGL(k_imax, dim3((unsigned)((a.nodes + TPB - 1) / TPB)), dim3(TPB), 0, s, a, imax);
}
void launch_diag_field_energy(const Inst* d, int64_t ncell, double* acc, hipStream_t s) {
  int64_t nb = (ncell + TPB - 1) / TPB;
  nb = nb > 2048 ? 2048 : nb;
  hipLaunchKernelGGL(k_diag_field_energy, dim3((unsigned)nb), dim3(TPB), 0, s, d, ncell, acc);
}
void launch_diag_deposit(const Inst* d, int D, int order, int capacity, double* grid, int what,
                         hipStream_t s) {
  unsigned nb = (unsigned)((capacity + TPB - 1) / TPB);
  nb = nb < 1 ? 1 : (nb > 4096 ? 4096 : nb);
  if (order == 1) {
    DISPATCH_D(D, hipLaunchKernelGGL((k_diag_deposit<DD, 1>), dim3(nb), dim3(TPB), 0, s, d, grid, what));
  } else {
    DISPATCH_D(D, hipLaunchKernelGGL((k_diag_deposit<DD, 2>), dim3(nb), dim3(TPB), 0, s, d, grid, what));
  }
}
void launch_diag_gauss(const Inst* d, int D, const double* rho, double* acc, hipStream_t s) {
  DISPATCH_D(D, hipLaunchKernelGGL((k_diag_gauss<DD>), dim3(2048), dim3(TPB), 0, s, d, rho, acc));
}
void launch_table_probe(const TabHdr* tab, const float* A, float* P, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_table_probe, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tab, A, P, n);
}

}  // namespace pic
