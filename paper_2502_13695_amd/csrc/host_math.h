// Host-side FP64 math of the PIC library: canonical discrete problem, laser
// source, Keldysh rate (Sec. 2.1, Eq. 1-3) and its FP32 lookup table.
#pragma once

#include <vector>

#include "pic.h"
#include "pic_common.h"

namespace pic {

struct MatC {
  double gap_eV, n_index, n0, mred, mol_kg, e_kg, p_kg;
  float ie;                 // 1/eps_r (static) or 1/eps_inf (Lorentz)
  double lam0, gamma, eps_inf, deps;   // Lorentz pole (lam0 = 0: static)
  float lor[3];             // oscillator update (a, c, c deps); zeros when static
  double impact_P;          // impact-ionization rate constant [1/s] (0: none)
  double impact_th;         // its threshold energy [J]
  float chi3;               // Kerr chi3 = (4/3) n^2 eps0 c n2 [m^2/V^2] (0: linear)
};

// Von Neumann stability of the Yee update coupled to the explicit Lorentz
// oscillator (lossless medium), for the largest sum_d C_d^2 of the grid.
bool lorentz_stable(double ie, double c, double cd, double s2max);

struct Canon {
  int D;
  int64_t n[3];
  double dx[3];
  bool per[3];
  bool collide;   // binary collisions every step
  bool impact;    // impact ionization (some material has a rate constant)
  double dt;
  float C[3], kmur[3];
  int nwin;
  int nmat;
  MatC mats[MAXMAT];
  double vcell;
  int ppc;
  // laser
  double lam, omega, fwhm, t0, T, waist, cep, I0, E0, env2;
  int env, pol;
  std::vector<signed char> mat_cell;   // per cell x index
  std::vector<signed char> mat_node;   // per node x index
};

pic_status canonicalize(const pic_config* cfg, Canon* out);
double laser_field(const Canon& c, double t);
double transverse_profile(const Canon& c, double y, double z);

// Keldysh volumetric rate W(A) [m^-3 s^-1], FP64, `terms` terms of Eq. (3).
// The series stops once a bound of its tail is below 2^-tol_bits of the sum.
double keldysh_W(const MatC& m, double lam, int terms, double A, int tol_bits = 60);

struct TableHost {
  std::vector<unsigned char> bytes;   // TabHdr, TabSeg[], coefficients
  float acut = 0.f, asat = 0.f;
};
// Table of P(A) = 1 - exp(-W dt / n0) for material `mat`.
pic_status build_table(const Canon& c, int mat, int terms, TableHost* out, int tol_bits = 60);

}  // namespace pic
