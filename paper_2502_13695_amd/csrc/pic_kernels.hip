// Device kernels of the MI355X laser-dielectric PIC hot path.
//
// Per step (state E^n, b^n = cB^n, particles x^n with u^{n-1/2}):
//   push      gather E^n, b^n with the particle shape, relativistic Boris,
//             move, Esirkepov deposit of J^{n+1/2} (global FP32 atomics)
//   bhalf     b^{n+1/2} = b^n - (1/2) C curl E^n
//   efull     E^{n+1} = E^n + (1/eps_r)(C curl b^{n+1/2} - dt J / eps0) with the
//             first-order outflow (Mur) chain on the faces and the laser
//             injected at x_min; J cleared for the next deposit
//   bhalf     b^{n+1} = b^{n+1/2} - (1/2) C curl E^{n+1}
//   amp       node |E^{n+1}| into the one-cycle window, exact sliding maximum
//             (van Herk / Gil-Werman blocks), amplitude A (Sec. 2.1)
//   ionize    per alive neutral: A at the neutral (shape gather), P from the
//             FP32 Keldysh table (Sec. 2.1), Philox draw, electron and
//             positive-carrier birth (Sec. 2.1, 3.2)
//   advance   step counter + 1
#include <hip/hip_runtime.h>

#include "pic_kernels.h"

namespace pic {

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ int find_inst(const Group& g) {
  const int b = blockIdx.x;
  int lo = 0, hi = g.n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (g.off[mid] <= b) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int wrapi(int j, int n, int per) {
  if (!per) return j;
  return j < 0 ? j + n : (j >= n ? j - n : j);
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
__device__ __forceinline__ float gather(const float* __restrict__ F, const Axis<ORDER>& X,
                                        const Axis<ORDER>& Y, const Axis<ORDER>& Z, int hx, int hy,
                                        int hz) {
  constexpr int SY = D >= 2 ? ORDER + 1 : 1;
  constexpr int SZ = D >= 3 ? ORDER + 1 : 1;
  float acc = 0.0f;
#pragma unroll
  for (int c = 0; c < SZ; ++c) {
    const float wz = D >= 3 ? (hz ? Z.wh[c] : Z.wn[c]) : 1.0f;
    const int oz = D >= 3 ? (hz ? Z.oh[c] : Z.on[c]) : 0;
#pragma unroll
    for (int b = 0; b < SY; ++b) {
      const float wy = D >= 2 ? (hy ? Y.wh[b] : Y.wn[b]) : 1.0f;
      const int oy = D >= 2 ? (hy ? Y.oh[b] : Y.on[b]) : 0;
      float row = 0.0f;
#pragma unroll
      for (int a = 0; a <= ORDER; ++a) {
        const float wx = hx ? X.wh[a] : X.wn[a];
        const int ox = hx ? X.oh[a] : X.on[a];
        row += wx * F[ox + oy + oz];
      }
      acc += wz * wy * row;
    }
  }
  return acc;
}

// Esirkepov local arrays along one axis: L = 5 (order 2) or 4 (order 1)
// nodes starting at `org`; S0 and DS = S1 - S0; [lo, hi) = nonzero range.
template <int ORDER>
struct Esk {
  static constexpr int L = ORDER == 2 ? 5 : 4;
  float S0[L], DS[L];
  int org, lo, hi;
};

template <int ORDER>
__device__ __forceinline__ void esk_axis(Esk<ORDER>& e, int c0, float t0, int c1, float t1) {
  float w0[ORDER + 1], w1[ORDER + 1];
  const int b0 = shape<ORDER>(c0, t0, 0, w0);
  const int b1 = shape<ORDER>(c1, t1, 0, w1);
  constexpr int L = Esk<ORDER>::L;
  e.org = b0 - 1;   // S0 occupies local 1 .. ORDER + 1
  const int sh = b1 - b0;   // -1, 0, 1
#pragma unroll
  for (int q = 0; q < L; ++q) e.S0[q] = 0.0f;
#pragma unroll
  for (int q = 0; q <= ORDER; ++q) e.S0[q + 1] = w0[q];
#pragma unroll
  for (int q = 0; q < L; ++q) {
    const int r = q - 1 - sh;
    const float s1 = (r >= 0 && r <= ORDER) ? w1[r] : 0.0f;
    e.DS[q] = s1 - e.S0[q];
  }
  e.lo = sh < 0 ? 0 : 1;
  e.hi = sh > 0 ? ORDER + 3 : ORDER + 2;
}

template <int D, int ORDER>
__global__ __launch_bounds__(TPB) void k_push(Group g) {
  const int ii = find_inst(g);
  const Inst& I = g.insts[ii];
  const int nthr = (g.off[ii + 1] - g.off[ii]) * TPB;
  const int tid = (blockIdx.x - g.off[ii]) * TPB + threadIdx.x;
  int count = *I.pcount;
  count = count < I.capacity ? count : I.capacity;
  for (int p = tid; p < count; p += nthr) {
    const uint8_t kind = I.pkind[p];
    if (kind == DEAD) continue;
    int ci, cj, ck;
    unpack_cell(D, I.pcell[p], ci, cj, ck);
    const float t0 = I.po0[p];
    const float t1 = D >= 2 ? I.po1[p] : 0.0f;
    const float t2 = D >= 3 ? I.po2[p] : 0.0f;
    float ux = I.pu0[p], uy = I.pu1[p], uz = I.pu2[p];
    // ---- gather E^n, b^n
    Axis<ORDER> X, Y, Z;
    make_axis<ORDER>(X, ci, t0, I.nx, 0, G, 1);
    if (D >= 2) make_axis<ORDER>(Y, cj, t1, I.ny, I.per_y, I.Gy, I.sy);
    if (D >= 3) make_axis<ORDER>(Z, ck, t2, I.nz, I.per_z, I.Gz, I.sz);
    const float ex = gather<D, ORDER>(I.E0, X, Y, Z, 1, 0, 0);
    const float ey = gather<D, ORDER>(I.E1, X, Y, Z, 0, 1, 0);
    const float ez = gather<D, ORDER>(I.E2, X, Y, Z, 0, 0, 1);
    const float bx = gather<D, ORDER>(I.B0, X, Y, Z, 0, 1, 1);
    const float by = gather<D, ORDER>(I.B1, X, Y, Z, 1, 0, 1);
    const float bz = gather<D, ORDER>(I.B2, X, Y, Z, 1, 1, 0);
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
    const float ig = 1.0f / sqrtf(1.0f + ux * ux + uy * uy + uz * uz);
    // ---- move: integer cell + FP32 offset, at most one cell per step
    int dead = 0;
    int ni = ci, nj = cj, nk = ck;
    float n0 = t0, n1 = t1, n2 = t2;
    auto move = [&](float& t, int& c, float disp) {
      float xn = t + disp;
      if (xn >= 1.0f) {
        xn -= 1.0f;
        c += 1;
      } else if (xn < 0.0f) {
        xn += 1.0f;
        c -= 1;
        if (xn >= 1.0f) { xn = 0.0f; c += 1; }
      }
      t = xn;
    };
    move(n0, ni, I.C[0] * ux * ig);
    if (D >= 2) move(n1, nj, I.C[1] * uy * ig);
    if (D >= 3) move(n2, nk, I.C[2] * uz * ig);
    // ---- Esirkepov deposit of J^{n+1/2} (scaled: dt J / eps0, V/m)
    Esk<ORDER> ex_, ey_, ez_;
    esk_axis<ORDER>(ex_, ci, t0, ni, n0);
    if (D >= 2) esk_axis<ORDER>(ey_, cj, t1, nj, n1);
    if (D >= 3) esk_axis<ORDER>(ez_, ck, t2, nk, n2);
    constexpr int L = Esk<ORDER>::L;
    constexpr int LY = D >= 2 ? L : 1;
    constexpr int LZ = D >= 3 ? L : 1;
    const float qx = I.kq[kind][0], qy = I.kq[kind][1], qz = I.kq[kind][2];
    const int ylo = D >= 2 ? ey_.lo : 0, yhi = D >= 2 ? ey_.hi : 1;
    const int zlo = D >= 3 ? ez_.lo : 0, zhi = D >= 3 ? ez_.hi : 1;
    for (int c = zlo; c < zhi; ++c) {
      const float s0z = D >= 3 ? ez_.S0[c] : 1.0f, dsz = D >= 3 ? ez_.DS[c] : 0.0f;
      const int oz = D >= 3 ? I.sz * (wrapi(ez_.org + c, I.nz, I.per_z) + I.Gz) : 0;
      for (int b = ylo; b < yhi; ++b) {
        const float s0y = D >= 2 ? ey_.S0[b] : 1.0f, dsy = D >= 2 ? ey_.DS[b] : 0.0f;
        const int oy = D >= 2 ? I.sy * (wrapi(ey_.org + b, I.ny, I.per_y) + I.Gy) : 0;
        // Jx: cumulative sum of Wx along x
        const float wbx = s0y * s0z + 0.5f * dsy * s0z + 0.5f * s0y * dsz + (1.0f / 3.0f) * dsy * dsz;
        float acc = 0.0f;
        for (int a = ex_.lo; a < ex_.hi - 1; ++a) {
          acc += ex_.DS[a] * wbx;
          const int ox = ex_.org + a + G;
          unsafeAtomicAdd(I.J0 + ox + oy + oz, -qx * acc);
        }
      }
    }
    // Jy
    {
      for (int c = zlo; c < zhi; ++c) {
        const float s0z = D >= 3 ? ez_.S0[c] : 1.0f, dsz = D >= 3 ? ez_.DS[c] : 0.0f;
        const int oz = D >= 3 ? I.sz * (wrapi(ez_.org + c, I.nz, I.per_z) + I.Gz) : 0;
        for (int a = ex_.lo; a < ex_.hi; ++a) {
          const float s0x = ex_.S0[a], dsx = ex_.DS[a];
          const float wby = s0x * s0z + 0.5f * dsx * s0z + 0.5f * s0x * dsz + (1.0f / 3.0f) * dsx * dsz;
          const int ox = ex_.org + a + G;
          if (D >= 2) {
            float acc = 0.0f;
            for (int b = ey_.lo; b < ey_.hi - 1; ++b) {
              acc += ey_.DS[b] * wby;
              const int oy = I.sy * (wrapi(ey_.org + b, I.ny, I.per_y) + I.Gy);
              unsafeAtomicAdd(I.J1 + ox + oy + oz, -qy * acc);
            }
          } else {
            unsafeAtomicAdd(I.J1 + ox, qy * uy * ig * wby);
          }
        }
      }
    }
    // Jz
    {
      for (int b = ylo; b < yhi; ++b) {
        const float s0y = D >= 2 ? ey_.S0[b] : 1.0f, dsy = D >= 2 ? ey_.DS[b] : 0.0f;
        const int oy = D >= 2 ? I.sy * (wrapi(ey_.org + b, I.ny, I.per_y) + I.Gy) : 0;
        for (int a = ex_.lo; a < ex_.hi; ++a) {
          const float s0x = ex_.S0[a], dsx = ex_.DS[a];
          const float wbz = s0x * s0y + 0.5f * dsx * s0y + 0.5f * s0x * dsy + (1.0f / 3.0f) * dsx * dsy;
          const int ox = ex_.org + a + G;
          if (D >= 3) {
            float acc = 0.0f;
            for (int c = ez_.lo; c < ez_.hi - 1; ++c) {
              acc += ez_.DS[c] * wbz;
              const int oz = I.sz * (wrapi(ez_.org + c, I.nz, I.per_z) + I.Gz);
              unsafeAtomicAdd(I.J2 + ox + oy + oz, -qz * acc);
            }
          } else {
            unsafeAtomicAdd(I.J2 + ox + oy, qz * uz * ig * wbz);
          }
        }
      }
    }
    (void)LY;
    (void)LZ;
    // ---- boundaries: outflow removes, periodic wraps
    if (ni < 0 || ni >= I.nx) dead = 1;
    if (D >= 2) {
      if (I.per_y) nj = wrapi(nj, I.ny, 1);
      else if (nj < 0 || nj >= I.ny) dead = 1;
    }
    if (D >= 3) {
      if (I.per_z) nk = wrapi(nk, I.nz, 1);
      else if (nk < 0 || nk >= I.nz) dead = 1;
    }
    if (dead) {
      I.pkind[p] = DEAD;
      continue;
    }
    I.pcell[p] = pack_cell(D, ni, nj, nk);
    I.po0[p] = n0;
    if (D >= 2) I.po1[p] = n1;
    if (D >= 3) I.po2[p] = n2;
    I.pu0[p] = ux;
    I.pu1[p] = uy;
    I.pu2[p] = uz;
  }
}

// ------------------------------------------------------------ field solve
// decode a padded linear index into logical (i, j, k)
template <int D>
__device__ __forceinline__ void decode(const Inst& I, int64_t p, int& i, int& j, int& k) {
  const int ai = (int)(p % I.Px);
  const int64_t r = p / I.Px;
  const int aj = D >= 2 ? (int)(r % I.Py) : 0;
  const int ak = D >= 3 ? (int)(r / I.Py) : 0;
  i = ai - G;
  j = aj - I.Gy;
  k = ak - I.Gz;
}

// valid range of a staggered component along one present axis
__device__ __forceinline__ bool in_rng(int v, int n, int half, int per, int lo_node) {
  if (half || per) return v >= 0 && v < n;
  return v >= lo_node && v <= n - lo_node;
}

template <int D>
__global__ __launch_bounds__(TPB) void k_bhalf(Group g) {
  const int ii = find_inst(g);
  const Inst& I = g.insts[ii];
  const int64_t p = (int64_t)(blockIdx.x - g.off[ii]) * TPB + threadIdx.x;
  if (p >= (int64_t)I.Px * I.Py * I.Pz) return;
  int i, j, k;
  decode<D>(I, p, i, j, k);
  const float hx = I.halfC[0], hy = I.halfC[1], hz = I.halfC[2];
  // neighbour offsets (+1 along each axis, wrapped on periodic axes)
  const int dxp = 1;
  const int dyp = D >= 2 ? (I.per_y && j == I.ny - 1 ? -(I.ny - 1) * I.sy : I.sy) : 0;
  const int dzp = D >= 3 ? (I.per_z && k == I.nz - 1 ? -(I.nz - 1) * I.sz : I.sz) : 0;
  const bool yin_n = D < 2 || in_rng(j, I.ny, 0, I.per_y, 0), yin_h = D < 2 || in_rng(j, I.ny, 1, I.per_y, 0);
  const bool zin_n = D < 3 || in_rng(k, I.nz, 0, I.per_z, 0), zin_h = D < 3 || in_rng(k, I.nz, 1, I.per_z, 0);
  const bool xin_n = in_rng(i, I.nx, 0, 0, 0), xin_h = in_rng(i, I.nx, 1, 0, 0);
  // bx at (x node, y half, z half): -(dEz/dy - dEy/dz)
  if (xin_n && (D < 2 || yin_h) && (D < 3 || zin_h)) {
    float cu = 0.0f;
    if (D >= 2) cu += hy * (I.E2[p + dyp] - I.E2[p]);
    if (D >= 3) cu -= hz * (I.E1[p + dzp] - I.E1[p]);
    I.B0[p] -= cu;
  }
  // by at (x half, y node, z half): -(dEx/dz - dEz/dx)
  if (xin_h && yin_n && (D < 3 || zin_h)) {
    float cu = -hx * (I.E2[p + dxp] - I.E2[p]);
    if (D >= 3) cu += hz * (I.E0[p + dzp] - I.E0[p]);
    I.B1[p] -= cu;
  }
  // bz at (x half, y half, z node): -(dEy/dx - dEx/dy)
  if (xin_h && (D < 2 || yin_h) && zin_n) {
    float cu = hx * (I.E1[p + dxp] - I.E1[p]);
    if (D >= 2) cu -= hy * (I.E0[p + dyp] - I.E0[p]);
    I.B2[p] -= cu;
  }
}

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

template <int D>
__global__ __launch_bounds__(TPB) void k_efull(Group g) {
  const int ii = find_inst(g);
  const Inst& I = g.insts[ii];
  const int64_t p = (int64_t)(blockIdx.x - g.off[ii]) * TPB + threadIdx.x;
  if (p >= (int64_t)I.Px * I.Py * I.Pz) return;
  int i, j, k;
  decode<D>(I, p, i, j, k);
  const float jx = I.J0[p], jy = I.J1[p], jz = I.J2[p];
  I.J0[p] = 0.0f;
  I.J1[p] = 0.0f;
  I.J2[p] = 0.0f;
  const float Cx = I.C[0], Cy = I.C[1], Cz = I.C[2];
  const int ai = i + G;
  const int dym = D >= 2 ? (I.per_y && j == 0 ? (I.ny - 1) * I.sy : -I.sy) : 0;
  const int dzm = D >= 3 ? (I.per_z && k == 0 ? (I.nz - 1) * I.sz : -I.sz) : 0;
  // interior test per staggering (node axes exclude the outflow faces)
  const bool xh = in_rng(i, I.nx, 1, 0, 0), xn = in_rng(i, I.nx, 0, 0, 1);
  const bool yh = D < 2 || in_rng(j, I.ny, 1, I.per_y, 0);
  const bool yn = D < 2 || in_rng(j, I.ny, 0, I.per_y, 1);
  const bool zh = D < 3 || in_rng(k, I.nz, 1, I.per_z, 0);
  const bool zn = D < 3 || in_rng(k, I.nz, 0, I.per_z, 1);
  const int step = *I.step;
  // incident field factors for the x_min face
  float4 s0 = make_float4(0.f, 0.f, 0.f, 0.f), s1 = s0;
  if (i == 1) {
    if (step < I.nsrc) s0 = I.src[step];
    if (step + 1 < I.nsrc) s1 = I.src[step + 1];
  }
  // ---------------- Ex (x half, y node, z node)
  if (xh && yn && zn) {
    const float ie = I.ie_half[ai];
    float cu = 0.0f;
    if (D >= 2) cu += Cy * (I.B2[p] - I.B2[p + dym]);
    if (D >= 3) cu -= Cz * (I.B1[p] - I.B1[p + dzm]);
    const float old = I.E0[p];
    const float nw = old + ie * (cu - jx);
    I.E0[p] = nw;
    // faces: y (priority over z), then z, then the y-z edge
    if (D >= 2 && !I.per_y) {
      const int fy = (j == 1) ? -1 : (j == I.ny - 1 ? 1 : 0);
      const int fz = (D >= 3 && !I.per_z) ? ((k == 1) ? -1 : (k == I.nz - 1 ? 1 : 0)) : 0;
      const int oy = fy * I.sy, oz = fz * I.sz;
      float qz_new = 0.f, qz_old = 0.f;
      if (fz) {   // z-face point (x half, y interior): neighbour p
        qz_old = I.E0[p + oz];
        qz_new = mur(qz_old, old, nw, I.kmur[2]);
        I.E0[p + oz] = qz_new;
      }
      if (fy) {
        const float qo = I.E0[p + oy];
        I.E0[p + oy] = mur(qo, old, nw, I.kmur[1]);
        if (fz) {   // y-z edge: y priority, neighbour is the z-face point
          const float qe = I.E0[p + oy + oz];
          I.E0[p + oy + oz] = mur(qe, qz_old, qz_new, I.kmur[1]);
        }
      }
    } else if (D >= 3 && !I.per_z) {
      const int fz = (k == 1) ? -1 : (k == I.nz - 1 ? 1 : 0);
      if (fz) {
        const float qo = I.E0[p + fz * I.sz];
        I.E0[p + fz * I.sz] = mur(qo, old, nw, I.kmur[2]);
      }
    }
  }
  // ---------------- Ey (x node, y half, z node) and Ez (x node, y node, z half)
#pragma unroll
  for (int comp = 1; comp <= 2; ++comp) {
    const bool inside = comp == 1 ? (xn && yh && zn) : (xn && yn && zh);
    if (!inside) continue;
    float* E = comp == 1 ? I.E1 : I.E2;
    const float ie = I.ie_node[ai];
    float cu;
    if (comp == 1) {   // dbx/dz - dbz/dx
      cu = -Cx * (I.B2[p] - I.B2[p - 1]);
      if (D >= 3) cu += Cz * (I.B0[p] - I.B0[p + dzm]);
    } else {           // dby/dx - dbx/dy
      cu = Cx * (I.B1[p] - I.B1[p - 1]);
      if (D >= 2) cu -= Cy * (I.B0[p] - I.B0[p + dym]);
    }
    const float jj = comp == 1 ? jy : jz;
    const float old = E[p];
    const float nw = old + ie * (cu - jj);
    E[p] = nw;
    // transverse face this component is tangential to (z for Ey, y for Ez)
    const int td = comp == 1 ? 2 : 1;
    int ft = 0, st = 0;
    if (td == 1 && D >= 2 && !I.per_y) {
      ft = (j == 1) ? -1 : (j == I.ny - 1 ? 1 : 0);
      st = I.sy;
    }
    if (td == 2 && D >= 3 && !I.per_z) {
      ft = (k == 1) ? -1 : (k == I.nz - 1 ? 1 : 0);
      st = I.sz;
    }
    const int fx = (i == 1) ? -1 : (i == I.nx - 1 ? 1 : 0);
    float qt_new = 0.f, qt_old = 0.f;
    if (ft) {   // transverse-face point: neighbour p
      qt_old = E[p + ft * st];
      qt_new = mur(qt_old, old, nw, I.kmur[td]);
      E[p + ft * st] = qt_new;
    }
    if (fx) {   // x-face point (priority x): neighbour p; edge: neighbour is qt
      const bool inj = (fx < 0) && (comp == I.pol);
      const int tp = (j + I.Gy) + I.Py * (k + I.Gz);
      float prof = inj ? I.prof[tp] : 0.f;
      MurInc m{prof * s0.x, prof * s1.x, prof * s0.y, prof * s1.y};
      const float qo = E[p + fx];
      E[p + fx] = inj ? mur_inc(qo, old, nw, I.kmur[0], m) : mur(qo, old, nw, I.kmur[0]);
      if (ft) {
        const int te = tp + (td == 1 ? ft : ft * I.Py);
        float prof2 = inj ? I.prof[te] : 0.f;
        MurInc m2{prof2 * s0.x, prof2 * s1.x, prof2 * s0.y, prof2 * s1.y};
        const float qe = E[p + fx + ft * st];
        E[p + fx + ft * st] = inj ? mur_inc(qe, qt_old, qt_new, I.kmur[0], m2)
                                  : mur(qe, qt_old, qt_new, I.kmur[0]);
      }
    }
  }
}

// ------------------------------------------------------- amplitude window
template <int D>
__global__ __launch_bounds__(TPB) void k_amp(Group g) {
  const int ii = find_inst(g);
  const Inst& I = g.insts[ii];
  const int64_t w = (int64_t)(blockIdx.x - g.off[ii]) * TPB + threadIdx.x;
  if (w >= I.wsz) return;
  const int wi = (int)(w % I.wnx);
  const int64_t r = w / I.wnx;
  const int aj = D >= 2 ? (int)(r % I.Py) : 0;
  const int ak = D >= 3 ? (int)(r / I.Py) : 0;
  const int i = I.wx0 + wi - G, j = aj - I.Gy, k = ak - I.Gz;
  // window nodes inside the box only
  if (i < 0 || i > I.nx) return;
  if (D >= 2 && (j < 0 || j > (I.per_y ? I.ny - 1 : I.ny))) return;
  if (D >= 3 && (k < 0 || k > (I.per_z ? I.nz - 1 : I.nz))) return;
  const int64_t p = (int64_t)(I.wx0 + wi) + (int64_t)I.sy * aj + (int64_t)I.sz * ak;
  const int dym = D >= 2 ? (I.per_y && j == 0 ? (I.ny - 1) * I.sy : -I.sy) : 0;
  const int dzm = D >= 3 ? (I.per_z && k == 0 ? (I.nz - 1) * I.sz : -I.sz) : 0;
  const float ex = 0.5f * (I.E0[p - 1] + I.E0[p]);
  const float ey = D >= 2 ? 0.5f * (I.E1[p + dym] + I.E1[p]) : I.E1[p];
  const float ez = D >= 3 ? 0.5f * (I.E2[p + dzm] + I.E2[p]) : I.E2[p];
  const float m = sqrtf(ex * ex + ey * ey + ez * ez);
  if (!(m <= 3.0e38f)) atomicOr(I.health, HEALTH_NONFINITE);
  const int slot = *I.step % I.nwin;
  I.ring[(int64_t)slot * I.wsz + w] = m;
  const float pre = slot == 0 ? m : fmaxf(I.prefix[w], m);
  I.prefix[w] = pre;
  const float a = slot + 1 < I.nwin ? fmaxf(I.suffix[(int64_t)(slot + 1) * I.wsz + w], pre) : pre;
  I.A[p] = a;
  if (slot == I.nwin - 1) {   // block complete: suffix maxima for the next block
    float run = 0.0f;
    for (int q = I.nwin - 1; q >= 0; --q) {
      run = fmaxf(run, I.ring[(int64_t)q * I.wsz + w]);
      I.suffix[(int64_t)q * I.wsz + w] = run;
    }
  }
}

// ------------------------------------------------------------- ionization
__device__ __forceinline__ void maxwell(uint64_t seed, uint64_t id, uint32_t purpose, float sig,
                                        float& ux, float& uy, float& uz) {
  const u32x4 w = draw(seed, id, 0u, purpose);
  const float u1 = (float)(((double)w.x + 0.5) * 0x1p-32);
  const float u2 = (float)(((double)w.y + 0.5) * 0x1p-32);
  const float u3 = (float)(((double)w.z + 0.5) * 0x1p-32);
  const float u4 = (float)(((double)w.w + 0.5) * 0x1p-32);
  const float r1 = sqrtf(-2.0f * logf(u1)), r2 = sqrtf(-2.0f * logf(u3));
  const float tp = 6.2831853071795864769f;
  ux = sig * r1 * cosf(tp * u2);
  uy = sig * r1 * sinf(tp * u2);
  uz = sig * r2 * cosf(tp * u4);
}

template <int D>
__device__ __forceinline__ uint64_t neutral_id(const Inst& I, int64_t jn, int& ci, int& cj, int& ck) {
  const int64_t m = jn / I.ppc;
  const int64_t kk = jn - m * I.ppc;
  unpack_cell(D, I.mcell[m], ci, cj, ck);
  const int64_t lin = ci + (int64_t)I.nx * (cj + (int64_t)I.ny * ck);
  return (uint64_t)(lin * I.ppc + kk);
}

template <int D, int ORDER>
__global__ __launch_bounds__(TPB) void k_ionize(Group g) {
  const int ii = find_inst(g);
  const Inst& I = g.insts[ii];
  const int64_t jn = (int64_t)(blockIdx.x - g.off[ii]) * TPB + threadIdx.x;
  if (jn >= I.nneut) return;
  if (!((I.alive[jn >> 5] >> (jn & 31)) & 1u)) return;
  int ci, cj, ck;
  const uint64_t id = neutral_id<D>(I, jn, ci, cj, ck);
  const float t0 = I.no0[jn];
  const float t1 = D >= 2 ? I.no1[jn] : 0.f;
  const float t2 = D >= 3 ? I.no2[jn] : 0.f;
  // amplitude at the neutral: node-shape gather of A
  Axis<ORDER> X, Y, Z;
  make_axis<ORDER>(X, ci, t0, I.nx, 0, G, 1);
  if (D >= 2) make_axis<ORDER>(Y, cj, t1, I.ny, I.per_y, I.Gy, I.sy);
  if (D >= 3) make_axis<ORDER>(Z, ck, t2, I.nz, I.per_z, I.Gz, I.sz);
  const float Ap = gather<D, ORDER>(I.A, X, Y, Z, 0, 0, 0);
  const int mat = I.mat_cell[ci];
  if (mat < 0 || !(Ap >= I.acut[mat])) return;
  const float P = table_lookup(I.tab[mat], Ap);
  const int n1 = *I.step + 1;
  const u32x4 w = draw(I.seed, id, (uint32_t)n1, PURPOSE_IONIZE);
  // event iff (w + 1/2) 2^-32 < P, decided exactly in FP64
  if (!((double)w.x + 0.5 < (double)P * 4294967296.0)) return;
  atomicAnd(&I.alive[jn >> 5], ~(1u << (jn & 31)));
  I.death[jn] = n1;
  atomicAdd(&I.nevents[mat], 1ull);
  const int slot = atomicAdd(I.pcount, 2);
  if (slot + 2 > I.capacity) {
    atomicOr(I.health, HEALTH_CAPACITY);
    return;
  }
  float ux, uy, uz;
  maxwell(I.seed, id, PURPOSE_VEL, I.ksig[mat], ux, uy, uz);
  const uint32_t pc = pack_cell(D, ci, cj, ck);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int q = slot + s;
    I.pcell[q] = pc;
    I.po0[q] = t0;
    if (D >= 2) I.po1[q] = t1;
    if (D >= 3) I.po2[q] = t2;
    I.pu0[q] = ux;
    I.pu1[q] = uy;
    I.pu2[q] = uz;
    I.pkind[q] = (uint8_t)(2 * mat + s);
  }
}

__global__ void k_advance(const Inst* insts, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) *insts[i].step += 1;
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
    I.po0[q] = I.no0[jn];
    if (D >= 2) I.po1[q] = I.no1[jn];
    if (D >= 3) I.po2[q] = I.no2[jn];
    I.pu0[q] = ux;
    I.pu1[q] = uy;
    I.pu2[q] = uz;
    I.pkind[q] = (uint8_t)(2 * mat + s);
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

__global__ __launch_bounds__(TPB) void k_diag_field_energy(const Inst* d, int64_t ncell, double* acc) {
  const Inst& I = *d;
  double s = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * TPB + threadIdx.x; p < ncell; p += (int64_t)gridDim.x * TPB) {
    const int ai = (int)(p % I.Px);
    const double ex = I.E0[p], ey = I.E1[p], ez = I.E2[p];
    s += ex * ex / I.ie_half[ai] + (ey * ey + ez * ez) / I.ie_node[ai];
    const double bx = I.B0[p], by = I.B1[p], bz = I.B2[p];
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
    make_axis<ORDER>(X, ci, I.po0[p], I.nx, 0, G, 1);
    if (D >= 2) make_axis<ORDER>(Y, cj, I.po1[p], I.ny, I.per_y, I.Gy, I.sy);
    if (D >= 3) make_axis<ORDER>(Z, ck, I.po2[p], I.nz, I.per_z, I.Gz, I.sz);
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
  double mres = 0.0, mrho = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * TPB + threadIdx.x; p < ncell; p += (int64_t)gridDim.x * TPB) {
    int i, j, k;
    decode<D>(I, p, i, j, k);
    if (i < 1 || i > I.nx - 1) continue;
    if (D >= 2 && (I.per_y ? (j < 0 || j >= I.ny) : (j < 1 || j > I.ny - 1))) continue;
    if (D >= 3 && (I.per_z ? (k < 0 || k >= I.nz) : (k < 1 || k > I.nz - 1))) continue;
    const int ai = i + G;
    double div = ((double)I.E0[p] / I.ie_half[ai] - (double)I.E0[p - 1] / I.ie_half[ai - 1]) / I.dx[0];
    if (D >= 2) {
      const int dym = I.per_y && j == 0 ? (I.ny - 1) * I.sy : -I.sy;
      div += ((double)I.E1[p] - (double)I.E1[p + dym]) / I.ie_node[ai] / I.dx[1];
    }
    if (D >= 3) {
      const int dzm = I.per_z && k == 0 ? (I.nz - 1) * I.sz : -I.sz;
      div += ((double)I.E2[p] - (double)I.E2[p + dzm]) / I.ie_node[ai] / I.dx[2];
    }
    mres = fmax(mres, fabs(div - rho[p]));
    mrho = fmax(mrho, fabs(rho[p]));
  }
  atomicMax(reinterpret_cast<unsigned long long*>(acc), __double_as_longlong(mres));
  atomicMax(reinterpret_cast<unsigned long long*>(acc) + 1, __double_as_longlong(mrho));
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

void launch_push(const Group& g, int D, int order, hipStream_t s) {
  if (order == 1) {
    DISPATCH_D(D, hipLaunchKernelGGL((k_push<DD, 1>), dim3(g.blocks), dim3(TPB), 0, s, g));
  } else {
    DISPATCH_D(D, hipLaunchKernelGGL((k_push<DD, 2>), dim3(g.blocks), dim3(TPB), 0, s, g));
  }
}
void launch_bhalf(const Group& g, int D, hipStream_t s) {
  DISPATCH_D(D, hipLaunchKernelGGL((k_bhalf<DD>), dim3(g.blocks), dim3(TPB), 0, s, g));
}
void launch_efull(const Group& g, int D, hipStream_t s) {
  DISPATCH_D(D, hipLaunchKernelGGL((k_efull<DD>), dim3(g.blocks), dim3(TPB), 0, s, g));
}
void launch_amp(const Group& g, int D, hipStream_t s) {
  DISPATCH_D(D, hipLaunchKernelGGL((k_amp<DD>), dim3(g.blocks), dim3(TPB), 0, s, g));
}
void launch_ionize(const Group& g, int D, int order, hipStream_t s) {
  if (order == 1) {
    DISPATCH_D(D, hipLaunchKernelGGL((k_ionize<DD, 1>), dim3(g.blocks), dim3(TPB), 0, s, g));
  } else {
    DISPATCH_D(D, hipLaunchKernelGGL((k_ionize<DD, 2>), dim3(g.blocks), dim3(TPB), 0, s, g));
  }
}
void launch_advance(const Inst* insts, int n, hipStream_t s) {
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
