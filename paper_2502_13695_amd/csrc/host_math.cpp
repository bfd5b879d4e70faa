// Host-side FP64 math: canonical discrete problem (Sec. 3.1 time step, Table 1
// materials, Sec. 2.3 geometry, Sec. 3 pulse), the Keldysh rate of Sec. 2.1
// (Eq. 1-3) and the FP32 lookup table the ionization kernel reads.
// Compiled without floating-point contraction so the canonical coefficients
// are reproducible bit for bit.
#include "host_math.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace pic {

namespace {

constexpr double kC = 299792458.0;
constexpr double kQE = 1.602176634e-19;
constexpr double kME = 9.1093837015e-31;
constexpr double kEPS0 = 8.8541878128e-12;
constexpr double kHBAR = 1.054571817e-34;
constexpr double kNA = 6.02214076e23;
constexpr double kAMU = 1.66053906660e-27;
constexpr double kPI = 3.14159265358979323846;

float f32_down(double v) {
  float f = (float)v;
  if ((double)f > v) f = std::nextafter(f, -INFINITY);
  return f;
}

int material_at(const pic_config* cfg, double x) {
  for (int l = 0; l < cfg->nlayer; ++l) {
    const pic_layer& L = cfg->layers[l];
    if (L.lo_m <= x && x < L.hi_m) return L.material;
  }
  return -1;
}

// ---- complete elliptic integrals by the AGM (Abramowitz & Stegun 17.6);
// m is the parameter, m1 = 1 - m passed separately (no cancellation).
void ellipKE(double m, double m1, double* K, double* E) {
  double a = 1.0, b = std::sqrt(m1), acc = 0.5 * m, w = 1.0;
  for (int it = 0; it < 60; ++it) {
    const double c = 0.5 * (a - b);
    const double an = 0.5 * (a + b);
    b = std::sqrt(a * b);
    a = an;
    acc += w * c * c;
    w *= 2.0;
    if (std::fabs(c) <= 4e-16 * a) break;
  }
  *K = kPI / (2.0 * a);
  *E = *K * (1.0 - acc);
}

// ---- Dawson integral (Rybicki 1989, step 0.2; Maclaurin series near 0)
double dawson(double z) {
  const double az = std::fabs(z);
  if (az < 0.2) {
    const double z2 = z * z;
    double t = z, s = z;
    for (int k = 1; k < 14; ++k) {
      t *= -2.0 * z2 / (2 * k + 1);
      s += t;
    }
    return s;
  }
  static double ck[35];
  static bool init = false;
  if (!init) {
    for (int k = 1; k < 35; k += 2) ck[k] = std::exp(-(0.2 * k) * (0.2 * k));
    init = true;
  }
  const double h = 0.2;
  const double n0 = 2.0 * std::nearbyint(0.5 * az / h);
  const double xp = az - n0 * h;
  const double e1 = std::exp(2.0 * xp * h), e2 = e1 * e1;
  double ek = e1, s = 0.0;
  for (int k = 1; k < 35; k += 2) {
    s += ck[k] * (ek / (n0 + k) + 1.0 / (ek * (n0 - k)));
    ek *= e2;
  }
  const double v = std::exp(-xp * xp) * s / std::sqrt(kPI);
  return z < 0 ? -v : v;
}

// Dawson(z)/z as a function of z^2 (entire); used where z -> 0.
double dawson_over_z(double z2) {
  if (z2 < 0.04) {
    double t = 1.0, s = 1.0;
    for (int k = 1; k < 14; ++k) {
      t *= -2.0 * z2 / (2 * k + 1);
      s += t;
    }
    return s;
  }
  const double z = std::sqrt(z2);
  return dawson(z) / z;
}

struct KP {
  double x, alpha, beta, pref;   // pref: Eq. (2) prefactor times sqrt(pi/(2 K(g2)))
};

KP kparts(const MatC& m, double lam, double A) {
  const double om = 2.0 * kPI * kC / lam;
  const double Dl = m.gap_eV * kQE;
  const double ms = m.mred * kME;
  const double g = om * std::sqrt(ms * Dl) / (kQE * A);
  const double gg = g * g;
  const double g2 = 1.0 / (1.0 + gg), g1 = gg / (1.0 + gg);
  double K1, E1, K2, E2;
  ellipKE(g1, g2, &K1, &E1);
  ellipKE(g2, g1, &K2, &E2);
  KP p;
  p.x = (2.0 / kPI) * (Dl / (kHBAR * om)) * E2 / std::sqrt(g1);
  p.alpha = kPI * (K1 - E1) / E2;
  p.beta = kPI * kPI / (2.0 * K2 * E2);
  p.pref = 2.0 * (2.0 * om / (9.0 * kPI)) * std::pow(ms * om / (kHBAR * std::sqrt(g1)), 1.5) *
           std::sqrt(kPI / (2.0 * K2));
  return p;
}

// sum_{n = n0}^{terms-1} exp(-n alpha) Dawson(sqrt(beta (d + n))), stopping once
// the bound of the remaining tail, max(Dawson) e^{-m alpha}/(1 - e^{-alpha}) from
// the next index m, is below 2^-tol_bits of the partial sum of the whole series
// (s_before: the terms below n0, counted in that test only)
double qseries(const KP& p, double d, int n0, int terms, int tol_bits, double s_before = 0.0) {
  const double q = std::exp(-p.alpha);
  const double tailf = 0.5410442246 / (-std::expm1(-p.alpha));
  const double tol = std::ldexp(1.0, -tol_bits);
  double s = 0.0, qn = std::exp(-n0 * p.alpha);
  for (int n = n0; n < terms; ++n) {
    const double a = p.beta * (d + n);
    s += qn * dawson(std::sqrt(a > 0 ? a : 0.0));
    qn *= q;
    if (qn * tailf < tol * (s_before + s)) break;
  }
  return s;
}

}  // namespace

double keldysh_W(const MatC& m, double lam, int terms, double A, int tol_bits) {
  const KP p = kparts(m, lam, A);
  const double N = std::floor(p.x + 1.0);
  return p.pref * std::exp(-N * p.alpha) * qseries(p, N - p.x, 0, terms, tol_bits);
}

pic_status canonicalize(const pic_config* cfg, Canon* c) {
  if (!cfg || !c) return PIC_E_INVAL;
  if (cfg->struct_size != sizeof(pic_config) || cfg->abi_version != PIC_ABI_VERSION)
    return PIC_E_VERSION;
  if (cfg->ndim < 1 || cfg->ndim > 3) return PIC_E_INVAL;
  if (cfg->nmat < 0 || cfg->nmat > MAXMAT || (cfg->nmat > 0 && !cfg->mats)) return PIC_E_INVAL;
  if (cfg->nlayer < 0 || (cfg->nlayer > 0 && !cfg->layers)) return PIC_E_INVAL;
  if (cfg->shape_order != 1 && cfg->shape_order != 2) return PIC_E_INVAL;
  if (cfg->ppc < 0 || !(cfg->cfl > 0 && cfg->cfl < 1)) return PIC_E_INVAL;
  if (cfg->keldysh_tol_bits < 0 || cfg->keldysh_tol_bits > 60) return PIC_E_INVAL;
  c->D = cfg->ndim;
  const int64_t maxn[3][3] = {{1 << 30, 1, 1}, {65535, 65535, 1}, {4095, 1023, 1023}};
  for (int d = 0; d < 3; ++d) {
    if (d < c->D) {
      if (cfg->n[d] < 4 || cfg->n[d] > maxn[c->D - 1][d] || !(cfg->dx_m[d] > 0)) return PIC_E_INVAL;
      c->n[d] = cfg->n[d];
      c->dx[d] = cfg->dx_m[d];
    } else {
      c->n[d] = 1;
      c->dx[d] = 1.0;
    }
    c->per[d] = (d > 0 && d < c->D && cfg->transverse_bc == PIC_BC_PERIODIC);
  }
  for (int l = 0; l < cfg->nlayer; ++l)
    if (cfg->layers[l].material < 0 || cfg->layers[l].material >= cfg->nmat) return PIC_E_INVAL;
  // time step: cfl / (c sqrt(sum 1/dx_d^2)), c dt / dx_0 rounded down to FP32
  double s = 0.0;
  for (int d = 0; d < c->D; ++d) s += 1.0 / (c->dx[d] * c->dx[d]);
  s = std::sqrt(s);
  const float c0 = f32_down(cfg->cfl / (c->dx[0] * s));
  c->dt = c0 * c->dx[0] / kC;
  for (int d = 0; d < 3; ++d) {
    c->C[d] = d < c->D ? (float)(c0 * (c->dx[0] / c->dx[d])) : 0.0f;
    if (d == 0) c->C[d] = c0;
    c->kmur[d] = d < c->D ? (float)((c->C[d] - 1.0) / (c->C[d] + 1.0)) : 0.0f;
  }
  const pic_laser& L = cfg->laser;
  if (!(L.lambda_m > 0) || !(L.fwhm_s > 0) || (L.pol_axis != 1 && L.pol_axis != 2)) return PIC_E_INVAL;
  c->lam = L.lambda_m;
  c->omega = 2.0 * kPI * kC / c->lam;
  c->nwin = (int)std::ceil((c->lam / kC) / c->dt);
  c->fwhm = L.fwhm_s;
  c->env = L.envelope;
  c->waist = L.waist_m;
  c->cep = L.cep_rad;
  c->pol = L.pol_axis;
  if (L.envelope == PIC_ENV_GAUSS) {
    c->t0 = L.t_peak_s > 0 ? L.t_peak_s : 3.0 * c->fwhm;
    c->T = 0.0;
    c->env2 = c->fwhm * std::sqrt(kPI / (4.0 * std::log(2.0)));
  } else if (L.envelope == PIC_ENV_SIN2) {
    c->T = c->fwhm / (1.0 - (2.0 / kPI) * std::asin(std::pow(2.0, -0.25)));
    c->t0 = L.t_peak_s > 0 ? L.t_peak_s : 0.5 * c->T;
    c->env2 = 3.0 * c->T / 8.0;
  } else {
    return PIC_E_INVAL;
  }
  c->I0 = L.fluence_Jcm2 > 0 ? L.fluence_Jcm2 * 1e4 / c->env2 : L.peak_Wcm2 * 1e4;
  c->E0 = std::sqrt(2.0 * c->I0 / (kC * kEPS0));
  c->nmat = cfg->nmat;
  c->impact = false;
  c->vcell = 1.0;
  for (int d = 0; d < c->D; ++d) c->vcell *= c->dx[d];
  c->ppc = cfg->ppc;
  if (cfg->collisions != 0 && cfg->collisions != 1) return PIC_E_INVAL;
  c->collide = cfg->collisions == 1;
  for (int m = 0; m < cfg->nmat; ++m) {
    const pic_material& M = cfg->mats[m];
    if (!(M.n_index > 0) || !(M.density_gcc > 0) || !(M.molar_mass_gmol > 0) || !(M.me_star > 0) ||
        !(M.mh_star > 0) || !(M.gap_eV > 0))
      return PIC_E_INVAL;
    MatC& mc = c->mats[m];
    mc.gap_eV = M.gap_eV;
    mc.n_index = M.n_index;
    mc.n0 = M.density_gcc * 1e6 / M.molar_mass_gmol * kNA;
    mc.mred = 1.0 / (1.0 / M.me_star + 1.0 / M.mh_star);
    mc.mol_kg = M.molar_mass_gmol * kAMU;
    mc.e_kg = M.me_star * kME;
    mc.p_kg = M.pos_mass_kg > 0 ? M.pos_mass_kg : mc.mol_kg;
    mc.lam0 = 0.0;
    mc.gamma = 0.0;
    mc.eps_inf = M.n_index * M.n_index;
    mc.deps = 0.0;
    mc.lor[0] = mc.lor[1] = mc.lor[2] = 0.0f;
    if (M.lorentz_lambda_m < 0) return PIC_E_INVAL;
    if (M.lorentz_lambda_m > 0) {
      // single pole: Re eps(omega_laser) = n^2 fixes deps; the oscillator is
      // centred at integer steps (a, c from the damping and the pole)
      if (!(M.eps_inf > 0) || !(M.lorentz_gamma_s >= 0)) return PIC_E_INVAL;
      const double w0 = 2.0 * kPI * kC / M.lorentz_lambda_m;
      const double w = c->omega;
      if (!(w0 > w)) return PIC_E_INVAL;
      const double g = M.lorentz_gamma_s;
      const double t = w0 * w0 - w * w;
      const double re_shape = w0 * w0 * t / (t * t + (g * w) * (g * w));
      const double deps = (M.n_index * M.n_index - M.eps_inf) / re_shape;
      if (deps < 0) return PIC_E_INVAL;
      const double den = 1.0 + 0.5 * g * c->dt;
      const double ca = (1.0 - 0.5 * g * c->dt) / den;
      const double cc = (w0 * c->dt) * (w0 * c->dt) / den;
      mc.lam0 = M.lorentz_lambda_m;
      mc.gamma = g;
      mc.eps_inf = M.eps_inf;
      mc.deps = deps;
      mc.lor[0] = (float)ca;
      mc.lor[1] = (float)cc;
      mc.lor[2] = (float)(cc * deps);
    }
    mc.ie = (float)(1.0 / mc.eps_inf);
    if (!(M.impact_rate_s >= 0)) return PIC_E_INVAL;
    mc.impact_P = M.impact_rate_s;
    {
      const double mu = M.me_star / M.mh_star;
      mc.impact_th = M.gap_eV * (1.0 + 2.0 * mu) / (1.0 + mu) * kQE;
    }
    if (mc.impact_P > 0) c->impact = true;
    if (!(M.kerr_n2_m2W >= 0)) return PIC_E_INVAL;
    mc.chi3 = (float)(4.0 / 3.0 * M.n_index * M.n_index * kEPS0 * kC * M.kerr_n2_m2W);
    if (M.lorentz_lambda_m > 0) {
      double s2max = 0.0;
      for (int d = 0; d < c->D; ++d) s2max += (double)c->C[d] * (double)c->C[d];
      if (!lorentz_stable(mc.ie, mc.lor[1], mc.lor[2], s2max)) return PIC_E_INVAL;
    }
  }
  const int64_t nx = c->n[0];
  c->mat_cell.assign(nx, -1);
  c->mat_node.assign(nx + 1, -1);
  for (int64_t i = 0; i < nx; ++i) c->mat_cell[i] = (signed char)material_at(cfg, ((double)i + 0.5) * c->dx[0]);
  for (int64_t i = 0; i <= nx; ++i) c->mat_node[i] = (signed char)material_at(cfg, (double)i * c->dx[0]);
  return PIC_OK;
}

// One mode of the coupled update gives, with w = z - 2 + 1/z,
//   f(w) = w^2 / ie + (c / ie + 4 s2 + c deps) w + 4 s2 c = 0;
// both roots are real and negative, and |z| = 1 needs them in [-4, 0]:
// f(-4) > 0 with the vertex above -4.  Both tests only tighten as s2 grows,
// so the grid's largest s2 = sum_d C_d^2 decides; c < 4 is the oscillator's
// own leapfrog bound.
bool lorentz_stable(double ie, double c, double cd, double s2max) {
  if (!(c >= 0.0 && c < 4.0)) return false;
  const double f4 = (16.0 - 4.0 * c) / ie - 4.0 * cd - s2max * (16.0 - 4.0 * c);
  return f4 > 0.0 && c / ie + 4.0 * s2max + cd <= 8.0 / ie;
}

double laser_field(const Canon& c, double t) {
  double env;
  if (c.env == PIC_ENV_GAUSS) {
    const double u = t - c.t0;
    env = std::exp(-2.0 * std::log(2.0) * u * u / (c.fwhm * c.fwhm));
  } else {
    const double s = t - c.t0 + 0.5 * c.T;
    const double sn = std::sin(kPI * s / c.T);
    env = (s >= 0 && s <= c.T) ? sn * sn : 0.0;
  }
  return c.E0 * env * std::cos(c.omega * (t - c.t0) + c.cep);
}

double transverse_profile(const Canon& c, double y, double z) {
  if (c.D == 1 || !(c.waist > 0)) return 1.0;
  return std::exp(-(y * y + z * z) / (c.waist * c.waist));
}

// --------------------------------------------------------------- the table
namespace {

struct Ctx {
  const MatC* m;
  double lam, dt;
  int terms, tol_bits;
};

double rate_r(const Ctx& k, double A) { return keldysh_W(*k.m, k.lam, k.terms, A, k.tol_bits) * k.dt / k.m->n0; }
double xof(const Ctx& k, double A) { return kparts(*k.m, k.lam, A).x; }

// One channel (floor(x+1) = N held fixed): r = pre [Dawson(sqrt(beta d)) + sum_{n>=1}],
// d = N - x.  Returns S1 = pre sum_{n>=1}, the n = 0 term T0, and the pieces
// needed for T0 / sqrt(A_k - A) near the closing.
struct Split {
  double S1, T0, pre, beta, d;
};

Split split_r(const Ctx& k, double A, double N) {
  const KP p = kparts(*k.m, k.lam, A);
  Split s;
  s.pre = p.pref * std::exp(-N * p.alpha) * k.dt / k.m->n0;
  s.d = N - p.x;
  s.beta = p.beta;
  const double t0 = dawson(std::sqrt(s.d > 0 ? p.beta * s.d : 0.0));
  // the n >= 1 part stops where the whole series would: the n = 0 term counts
  // in each stopping test, and the test after n = 0 alone may end the series
  const double tail1 = std::exp(-p.alpha) * (0.5410442246 / (-std::expm1(-p.alpha)));
  const bool stop0 = k.terms <= 1 || tail1 < std::ldexp(1.0, -k.tol_bits) * t0;
  s.S1 = stop0 ? 0.0 : s.pre * qseries(p, s.d, 1, k.terms, k.tol_bits, t0);
  s.T0 = s.pre * t0;
  return s;
}

// largest value of c0 + c1 f + c2 f^2 + c3 f^3 over [lo, hi]: the ends and
// the stationary points inside
double cubic_max(const double* c, double lo, double hi) {
  auto val = [&](double f) { return c[0] + f * (c[1] + f * (c[2] + f * c[3])); };
  double m = std::max(val(lo), val(hi));
  const double a = 3.0 * c[3], b = 2.0 * c[2], cc = c[1];   // derivative a f^2 + b f + cc
  if (a == 0.0) {
    if (b != 0.0) {
      const double f = -cc / b;
      if (f > lo && f < hi) m = std::max(m, val(f));
    }
    return m;
  }
  const double disc = b * b - 4.0 * a * cc;
  if (disc < 0.0) return m;
  const double sq = std::sqrt(disc);
  for (double f : {(-b - sq) / (2.0 * a), (-b + sq) / (2.0 * a)})
    if (f > lo && f < hi) m = std::max(m, val(f));
  return m;
}

// monomial coefficients of the cubic through (t_j, y_j), j = 0..3
void cubic_fit(const double* t, const double* y, double* c) {
  double M[4][5];
  for (int r = 0; r < 4; ++r) {
    double p = 1.0;
    for (int q = 0; q < 4; ++q) {
      M[r][q] = p;
      p *= t[r];
    }
    M[r][4] = y[r];
  }
  for (int col = 0; col < 4; ++col) {
    int piv = col;
    for (int r = col + 1; r < 4; ++r)
      if (std::fabs(M[r][col]) > std::fabs(M[piv][col])) piv = r;
    for (int q = 0; q < 5; ++q) std::swap(M[col][q], M[piv][q]);
    for (int r = 0; r < 4; ++r) {
      if (r == col) continue;
      const double f = M[r][col] / M[col][col];
      for (int q = col; q < 5; ++q) M[r][q] -= f * M[col][q];
    }
  }
  for (int r = 0; r < 4; ++r) c[r] = M[r][4] / M[r][r];
}

}  // namespace

pic_status build_table(const Canon& c, int mat, int terms, TableHost* out, int tol_bits) {
  if (mat < 0 || mat >= c.nmat || terms < 1 || tol_bits < 1 || tol_bits > 60) return PIC_E_INVAL;
  Ctx k{&c.mats[mat], c.lam, c.dt, terms, tol_bits};
  // 1. scan: amplitude cut (P < 2^-34 below) and saturation (r >= 40 above)
  const double Alo = 1e5, Ahi = 1e12, ratio = 1.0005;
  double acut = -1.0, asat = Ahi, prev = Alo;
  double xprev = -1.0;
  for (double A = Alo; A <= Ahi; A *= ratio) {
    const double x = xof(k, A);
    if (x < xprev) return PIC_E_DEVICE;   // x(A) must increase with A
    xprev = x;
    if (acut < 0) {
      const double r = rate_r(k, A);
      if (-std::expm1(-r) >= 0x1p-34) acut = prev;
    } else {
      // r increases steeply; test saturation every point once above the cut
      if (rate_r(k, A) >= 40.0) {
        asat = A;
        break;
      }
    }
    prev = A;
  }
  TableHost& T = *out;
  if (acut < 0) {   // never ionizes within the table range
    TabHdr h{INFINITY, INFINITY, 0, 0};
    T.bytes.assign(sizeof(TabHdr), 0);
    std::memcpy(T.bytes.data(), &h, sizeof h);
    T.acut = T.asat = INFINITY;
    return PIC_OK;
  }
  const float acut_f = f32_down(acut);
  float asat_f = (float)asat;
  if ((double)asat_f < asat) asat_f = std::nextafter(asat_f, INFINITY);
  // 2. channel closings x(A) = integer inside [acut, asat): FP32 breakpoints
  std::vector<float> bounds{acut_f};
  std::vector<double> exact{acut_f};   // exact closing A_k behind each FP32 bound
  const double xa = xof(k, acut_f), xb = xof(k, asat_f);
  for (double kk = std::floor(xa) + 1; kk <= xb; kk += 1.0) {
    double lo = acut_f, hi = asat_f;
    for (int it = 0; it < 200 && hi - lo > 1e-13 * hi; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (xof(k, mid) >= kk) hi = mid; else lo = mid;
    }
    float bf = (float)hi;
    while (xof(k, (double)bf) < kk) bf = std::nextafter(bf, INFINITY);
    while (true) {
      const float pb = std::nextafter(bf, 0.0f);
      if (xof(k, (double)pb) >= kk) bf = pb; else break;
    }
    if (bf > bounds.back() && bf < asat_f) {
      bounds.push_back(bf);
      exact.push_back(std::min(0.5 * (lo + hi), (double)bf));
    }
  }
  bounds.push_back(asat_f);
  exact.push_back(asat_f);
  const int nseg = (int)bounds.size() - 1;
  std::vector<TabSeg> segs(nseg);
  std::vector<float> recs;
  double running = 0.0;   // running maximum of the per-interval lookup bounds
  int base = 0;
  for (int s = 0; s < nseg; ++s) {
    const double lo = bounds[s], hi = bounds[s + 1];
    const double Ak = exact[s + 1];
    const bool sig = (s + 1 < nseg);   // right end is a channel closing
    const double N = std::floor(xof(k, lo) + 1.0);
    int nint = (int)std::ceil((hi - lo) / (2e-3 * lo));
    nint = std::max(nint, 4);
    const float inv_h = (float)(nint / (hi - lo));
    const double h = (hi - lo) / nint;
    // nodes are FP32 numbers: exact origins for the device's local coordinate
    std::vector<double> An(nint + 1), S1(nint + 1), S2(nint + 1);
    for (int j = 0; j <= nint; ++j) An[j] = (j == nint) ? hi : (double)(float)(lo + j * h);
    // dx/dA at the closing for the limit of T0 / sqrt(A_k - A)
    double xprime = 0.0;
    if (sig) {
      const double e = 1e-6 * Ak;
      xprime = (xof(k, Ak + e) - xof(k, Ak - e)) / (2.0 * e);
    }
    for (int j = 0; j <= nint; ++j) {
      const Split sp = split_r(k, An[j], N);
      if (!sig) {
        S1[j] = sp.S1 + sp.T0;
        S2[j] = 0.0;
        continue;
      }
      S1[j] = sp.S1;
      const double gap = Ak - An[j];
      // S2 = T0 / sqrt(A_k - A), smooth through A_k (d / (A_k - A) -> x'(A_k))
      double g = std::fabs(gap) > 1e-9 * Ak ? sp.d / gap : xprime;
      if (!(g > 0)) g = xprime;
      S2[j] = sp.pre * std::sqrt(sp.beta) * std::sqrt(g) * dawson_over_z(sp.beta * sp.d);
    }
    for (int i = 0; i < nint; ++i) {
      const int st = std::min(std::max(i - 1, 0), nint - 3);
      double t[4], y1[4], y2[4], c1[4], c2[4];
      for (int q = 0; q < 4; ++q) {
        t[q] = (An[st + q] - An[i]) * (double)inv_h;
        y1[q] = S1[st + q];
        y2[q] = S2[st + q];
      }
      cubic_fit(t, y1, c1);
      cubic_fit(t, y2, c2);
      float rec[TAB_REC] = {(float)An[i], (float)c1[0], (float)c1[1], (float)c1[2], (float)c1[3],
                            (float)c2[0], (float)c2[1], (float)c2[2], (float)c2[3], 0.f, 0.f, 0.f};
      // bound of the lookup over this interval, from the stored FP32
      // coefficients: the largest cubic value over a slightly widened local
      // coordinate range, plus the closing term at its largest distance
      const double fl = -1e-3, fh = 1.0 + 1e-3;
      const double q1[4] = {rec[1], rec[2], rec[3], rec[4]}, q2[4] = {rec[5], rec[6], rec[7], rec[8]};
      double rb = cubic_max(q1, fl, fh);
      double mag = std::fabs(q1[0]) + std::fabs(q1[1]) + std::fabs(q1[2]) + std::fabs(q1[3]);
      if (sig) {
        const double dmax = std::max(0.0, (hi - ((double)rec[0] + fl / (double)inv_h)) - (hi - Ak));
        const double m2 = std::max(0.0, cubic_max(q2, fl, fh));
        rb += std::sqrt(dmax) * m2;
        mag += std::sqrt(dmax) * (std::fabs(q2[0]) + std::fabs(q2[1]) + std::fabs(q2[2]) + std::fabs(q2[3]));
      }
      // FP32 evaluation of the Horner sums and of expm1f: a few ulp each
      rb = rb * (1.0 + 1e-5) + 1e-6 * mag;
      running = std::max(running, std::min(1.0, -std::expm1(-rb) * (1.0 + 1e-5)));
      float rf = (float)running;
      if ((double)rf < running) rf = std::nextafter(rf, INFINITY);
      rec[9] = rf;
      recs.insert(recs.end(), rec, rec + TAB_REC);
    }
    segs[s] = TabSeg{(float)lo, (float)hi, inv_h, base, nint, sig ? 1 : 0, (float)(hi - Ak), 0};
    base += nint;
  }
  TabHdr hdr{acut_f, asat_f, nseg, 0};
  T.bytes.resize(sizeof(TabHdr) + nseg * sizeof(TabSeg) + recs.size() * sizeof(float));
  unsigned char* p = T.bytes.data();
  std::memcpy(p, &hdr, sizeof hdr);
  std::memcpy(p + sizeof hdr, segs.data(), nseg * sizeof(TabSeg));
  std::memcpy(p + sizeof hdr + nseg * sizeof(TabSeg), recs.data(), recs.size() * sizeof(float));
  T.acut = acut_f;
  T.asat = asat_f;
  return PIC_OK;
}

}  // namespace pic
