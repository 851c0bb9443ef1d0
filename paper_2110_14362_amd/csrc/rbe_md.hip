// Langevin NPT integrator on gfx950 (section 3.2 eq. (24); appendix A eq.
// (99999); section 3.3 splitting B_V B_R A_V A_R O^p O A_R A_V | forces |
// B_R B_V), FP64.  Two kernels per step around the force evaluation:
//   k_md_first   every block replays the cell sub-steps (B_V, A_V, O^p, A_V:
//                scalar work, identical in every block) and applies B_R, A_R,
//                O, A_R to its particles; block 0 stores the mid-step cell
//   k_md_second  B_R on every particle, the kinetic tensor summed in a fixed
//                order by the last-arriving block, which forms the pressure
//                tensor and applies the closing B_V
// The start-of-step and mid-step cells live in two buffers, so no block reads
// a cell another block of the same launch writes.
//
// Rigid 3-site molecules: a thread owns a whole molecule.  Each position
// sub-flow (A_R) is followed by the position constraint solved in closed
// form (rigid_positions), with the momentum change the A_R map gives the
// position change, and each momentum sub-flow (B_R, O) by the projection of
// the molecule's momenta onto rigid-body motions (rigid_momenta).  The
// pressure takes the molecular form: centre-of-mass kinetic tensor and the
// atomic virial less sum sym((r - R_mol) F).
#include "rbe_md_internal.h"
#include <math.h>

// Multiply-adds are fused only where one source expression holds both, so the
// one-system and many-system kernels (the same code inlined in different
// surroundings) round identically.
#pragma clang fp contract(on)

namespace rbe {

__device__ __forceinline__ void philox_md(uint64_t c[4], uint64_t k0, uint64_t k1) {
  // Philox4x64-10 (Salmon et al., SC'11)
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    const uint64_t lo0 = M0 * c[0], hi0 = __umul64hi(M0, c[0]);
    const uint64_t lo1 = M1 * c[2], hi1 = __umul64hi(M1, c[2]);
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
  }
}

constexpr uint64_t kTagNoise = 0x6E6F6973ull;   // 'nois'
constexpr uint64_t kTagCell = 0x63656C6Cull;    // 'cell'

// three standard normals (Box-Muller on the four uniforms of one counter)
__device__ __forceinline__ void normals3(uint64_t seed, uint64_t sysid, uint64_t step,
                                         uint64_t index, uint64_t tag, double z[3]) {
  uint64_t c[4] = {step, index, tag, 0ull};
  philox_md(c, seed, sysid);
  double u[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) u[j] = (double)(c[j] >> 11) * 0x1.0p-53;
  const double a = sqrt(-2.0 * log(1.0 - u[0]));
  const double b = sqrt(-2.0 * log(1.0 - u[2]));
  double s1, c1, s3, c3;
  sincospi(2.0 * u[1], &s1, &c1);
  sincospi(2.0 * u[3], &s3, &c3);
  z[0] = a * c1; z[1] = a * s1; z[2] = b * c3;
}

// (e^{a h} - 1)/a, h at a = 0
__device__ __forceinline__ double expm1_over(double a, double h) {
  return a == 0.0 ? h : expm1(a * h) / a;
}

__device__ __forceinline__ double cell_volume(const MDCell& c) {
  if (c.mode == 2) return c.l[0] * c.l[1] * c.l[2];
  return c.mode == 0 ? c.V : c.A * c.L;
}

__device__ __forceinline__ void cell_rates(const MDCell& c, double a[3]) {
  if (c.mode == 0) {
    const double r = c.pV / (3.0 * c.M * c.V);
    a[0] = a[1] = a[2] = r;
  } else if (c.mode == 2) {
    for (int d = 0; d < 3; ++d) a[d] = c.pl[d] / (c.Ml[d] * c.l[d]);
  } else {
    a[0] = a[1] = c.pA / (2.0 * c.MA * c.A);
    a[2] = c.pL / (c.ML * c.L);
  }
}

__device__ __forceinline__ void cell_lengths(MDCell& c) {
  if (c.mode == 0) {
    const double L = cbrt(c.V);
    c.l[0] = c.asp[0] * L; c.l[1] = c.asp[1] * L; c.l[2] = c.asp[2] * L;
  } else if (c.mode == 2) {
    if (!(c.l[1] > 0.0)) c.err |= 1;
  } else {
    const double s = sqrt(c.A);
    c.l[0] = c.l[1] = s;
    c.l[2] = c.L;
  }
  if (!(c.l[0] > 0.0 && c.l[2] > 0.0)) c.err |= 1;    // collapsed or non-finite cell
}

__device__ __forceinline__ void B_V(const MDArgs& a, MDCell& c, double h) {
  const double P = a.ftm * a.P;
  const double* Pt = c.P_ins;
  if (c.mode == 0) c.pV += h * ((Pt[0] + Pt[1] + Pt[2]) / 3.0 - P);
  else if (c.mode == 2) {
    const double V = cell_volume(c);
    for (int d = 0; d < 3; ++d) c.pl[d] += h * V * (Pt[d] - P) / c.l[d];
  } else {
    c.pA += h * c.L * (0.5 * (Pt[0] + Pt[1]) - P);
    c.pL += h * c.A * (Pt[2] - P);
  }
}

__device__ __forceinline__ void A_V(MDCell& c, double h) {
  if (c.mode == 0) c.V += h * c.pV / c.M;
  else if (c.mode == 2) { for (int d = 0; d < 3; ++d) c.l[d] += h * c.pl[d] / c.Ml[d]; }
  else { c.A += h * c.pA / c.MA; c.L += h * c.pL / c.ML; }
}


// ---------------------------------------------------------------------------
// rigid 3-site molecules

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ __forceinline__ double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Mass-weighted orthogonal projection of the three momenta onto rigid-body
// motions, p_k <- m_k (P/M + w x rho_k), w = I^-1 L: the velocity stage of
// RATTLE for a rigid triangle in closed form (the part removed carries no
// linear or angular momentum, and no bond has a relative velocity along it
// afterwards).
// Divisions by the same value are multiplications by its reciprocal (an FP64
// division is a dozen dependent instructions; these chains run one molecule
// per lane), and every loop is unrolled so the arrays stay in registers.
__device__ __forceinline__ void rigid_momenta(const double r[3][3], double p[3][3], const double m[3],
                                              double iM) {
  double R[3], P[3], rho[3][3], L[3] = {0, 0, 0};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    R[d] = (m[0] * r[0][d] + m[1] * r[1][d] + m[2] * r[2][d]) * iM;
    P[d] = p[0][d] + p[1][d] + p[2][d];
  }
  double I[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
#pragma unroll
    for (int d = 0; d < 3; ++d) rho[k][d] = r[k][d] - R[d];
    double lk[3];
    cross3(rho[k], p[k], lk);
    const double r2 = dot3(rho[k], rho[k]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      L[d] += lk[d];
#pragma unroll
      for (int e = 0; e < 3; ++e) I[d][e] += m[k] * ((d == e ? r2 : 0.0) - rho[k][d] * rho[k][e]);
    }
  }
  // w = I^-1 L by the adjugate (I symmetric positive definite for a triangle)
  const double c00 = I[1][1] * I[2][2] - I[1][2] * I[2][1];
  const double c01 = I[1][2] * I[2][0] - I[1][0] * I[2][2];
  const double c02 = I[1][0] * I[2][1] - I[1][1] * I[2][0];
  const double c11 = I[0][0] * I[2][2] - I[0][2] * I[2][0];
  const double c12 = I[0][1] * I[2][0] - I[0][0] * I[2][1];
  const double c22 = I[0][0] * I[1][1] - I[0][1] * I[1][0];
  const double idet = 1.0 / (I[0][0] * c00 + I[0][1] * c01 + I[0][2] * c02);
  const double w[3] = {(c00 * L[0] + c01 * L[1] + c02 * L[2]) * idet,
                       (c01 * L[0] + c11 * L[1] + c12 * L[2]) * idet,
                       (c02 * L[0] + c12 * L[1] + c22 * L[2]) * idet};
  double V[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) V[d] = P[d] * iM;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double v[3];
    cross3(w, rho[k], v);
#pragma unroll
    for (int d = 0; d < 3; ++d) p[k][d] = m[k] * (V[d] + v[d]);
  }
}

// Position constraint in closed form.  r0: positions before the drift (a
// rigid molecule); r: unconstrained positions after it, replaced by the
// constrained ones.  The corrections of SHAKE (constraint forces along the
// old bonds) keep the centre of mass, lie in the old molecular plane (so each
// atom's coordinate along that plane's normal n is kept) and exert no torque
// about n with the old positions as lever arms.  The molecule's shape is
// fixed, so the result is a rotation of the reference triangle about the new
// centre of mass: its tilt follows from the three kept normal coordinates and
// its turn about n from the torque condition.  Returns false if no tilt
// matches (a drift far too long for the step).
__device__ __forceinline__ bool rigid_positions(const double r0[3][3], double r[3][3], const double m[3],
                                                double iM, double ra, double rb, double rc,
                                                double ira, double i2rc) {
  double b0[3], c0[3], Z[3], X[3], Y[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    b0[d] = r0[1][d] - r0[0][d];
    c0[d] = r0[2][d] - r0[0][d];
    X[d] = r0[2][d] - r0[1][d];
  }
  cross3(b0, c0, Z);
  const double izn = 1.0 / sqrt(dot3(Z, Z)), ixn = 1.0 / sqrt(dot3(X, X));
#pragma unroll
  for (int d = 0; d < 3; ++d) { Z[d] *= izn; X[d] *= ixn; }
  cross3(Z, X, Y);
  double D[3], C0[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    D[d] = (m[0] * r[0][d] + m[1] * r[1][d] + m[2] * r[2][d]) * iM;
    C0[d] = (m[0] * r0[0][d] + m[1] * r0[1][d] + m[2] * r0[2][d]) * iM;
  }
  double an[3][3], on[3][2];     // new (x, y, z) and old (x, y) in the frame
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double u[3], v[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) { u[d] = r[k][d] - D[d]; v[d] = r0[k][d] - C0[d]; }
    an[k][0] = dot3(u, X); an[k][1] = dot3(u, Y); an[k][2] = dot3(u, Z);
    on[k][0] = dot3(v, X); on[k][1] = dot3(v, Y);
  }
  // tilt: the unit vector t (reference frame) with t . c_k = normal coordinate
  const double ty = an[0][2] * ira;
  const double tx = (an[2][2] - an[1][2]) * i2rc;
  const double s2 = tx * tx + ty * ty;
  if (!(s2 < 1.0)) return false;
  const double tz = sqrt(1.0 - s2), sb = sqrt(s2);
  const double isb = sb > 0.0 ? 1.0 / sb : 0.0;
  const double cref[3][2] = {{0.0, ra}, {-rc, -rb}, {rc, -rb}};
  double q[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double cx = cref[k][0], cy = cref[k][1];
    if (sb > 0.0) {
      // rotation taking t to the normal, about the axis (ty, -tx, 0)/sb
      const double kx = ty * isb, ky = -tx * isb;
      const double kc = kx * cx + ky * cy;
      q[k][0] = cx * tz + kx * kc * (1.0 - tz);
      q[k][1] = cy * tz + ky * kc * (1.0 - tz);
      q[k][2] = (kx * cy - ky * cx) * sb;
    } else {
      q[k][0] = cx; q[k][1] = cy; q[k][2] = 0.0;
    }
  }
  // turn about the normal: sum_k m_k (o_k x p_k).n equals sum_k m_k (o_k x a_k).n
  double A = 0.0, B = 0.0, Lt = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    A += m[k] * (on[k][0] * q[k][0] + on[k][1] * q[k][1]);
    B += m[k] * (on[k][0] * q[k][1] - on[k][1] * q[k][0]);
    Lt += m[k] * (on[k][0] * an[k][1] - on[k][1] * an[k][0]);
  }
  const double sarg = Lt / sqrt(A * A + B * B);
  if (!(fabs(sarg) <= 1.0)) return false;
  const double th = asin(sarg) - atan2(B, A);
  double sn, cs;
  sincos(th, &sn, &cs);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double px = q[k][0] * cs - q[k][1] * sn;
    const double py = q[k][0] * sn + q[k][1] * cs;
    const double pz = q[k][2];
#pragma unroll
    for (int d = 0; d < 3; ++d) r[k][d] = D[d] + px * X[d] + py * Y[d] + pz * Z[d];
  }
  return true;
}

// A_R on a molecule, then the position constraint and the momentum change
// p += m (r_constrained - r_unconstrained) a / (e^{a h} - 1) per axis;
// e[d] = e^{a_d h}, f[d] = (e^{a_d h} - 1)/a_d, fi[d] = 1/f[d]; im[k] = 1/m[k]
__device__ __forceinline__ bool rigid_drift(const MDArgs& a, double r[3][3], double p[3][3],
                                            const double m[3], const double im[3], double iM,
                                            const double e[3], const double f[3], const double fi[3],
                                            double ira, double i2rc) {
  double r0[3][3], ru[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      r0[k][d] = r[k][d];
      ru[k][d] = r[k][d] * e[d] + p[k][d] * im[k] * f[d];
      r[k][d] = ru[k][d];
    }
  const bool ok = rigid_positions(r0, r, m, iM, a.ra, a.rb, a.rc, ira, i2rc);
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int d = 0; d < 3; ++d) p[k][d] += m[k] * (r[k][d] - ru[k][d]) * fi[d];
  return ok;
}

// atom index of free unit j (atoms outside the rigid block)
__device__ __forceinline__ int64_t free_atom(const MDArgs& a, int64_t j) {
  return j < a.rig_first ? j : j + 3 * a.rig_count;
}

// The sub-flow factors of one cell rate a over the half step h, the same
// for every particle: e^{-a h} and (e^{-a h} - 1)/(-a) (B_R), e^{a h} and
// (e^{a h} - 1)/a (each A_R).
struct MDFactors {
  double eB[3], fB[3], eA1[3], fA1[3], iA1[3], eA2[3], fA2[3], iA2[3];
};

// Block of k_md_first: kMdThreads units and four waves.  Waves 0-2 draw the
// noise of atom slot 0, 1, 2 of the block's units (an atom's counter is its
// index, so which lane draws it does not change the numbers); wave 3 replays
// the cell sub-steps in its first lane and forms the sub-flow factors in
// nine lanes; after the barrier wave 0 moves the units.  The units' chains
// no longer hold the noise and the exponentials, which are the same for
// every unit or independent of the unit's state.
__device__ __forceinline__ void md_first_body(const MDArgs& a, int bx) {
  __shared__ MDCell sc;
  __shared__ double rate[3][3];
  __shared__ MDFactors fac;
  __shared__ double zs[3][kMdThreads][3];
  const double h = 0.5 * a.dt;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t u = (int64_t)bx * kMdThreads + lane;
  const int64_t units = md_units(a);
  // wave 0 requests its unit's state first (the loads do not depend on the
  // cell or the noise); a free atom uses slot 0
  double r[3][3], p[3][3], F[3][3], m[3];
  const bool rig = u < a.rig_count;
  if (wave == 0 && u < units) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (k > 0 && !rig) break;
      const int64_t i = rig ? a.rig_first + 3 * u + k : free_atom(a, u - a.rig_count);
      m[k] = a.mass[i];
      r[k][0] = a.x[i]; r[k][1] = a.y[i]; r[k][2] = a.z[i];
      p[k][0] = a.px[i]; p[k][1] = a.py[i]; p[k][2] = a.pz[i];
      F[k][0] = a.fx[i]; F[k][1] = a.fy[i]; F[k][2] = a.fz[i];
    }
  }
  if (wave == 3) {
    // the cell state is copied word by word into LDS and replayed there by
    // one lane (a register copy of the whole struct went to scratch memory)
    constexpr int kCellWords = sizeof(MDCell) / 8;
    static_assert(sizeof(MDCell) % 8 == 0 && kCellWords <= 64, "cell copied by one wave");
    if (lane < kCellWords)
      reinterpret_cast<uint64_t*>(&sc)[lane] = reinterpret_cast<const uint64_t*>(a.cell_in)[lane];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane == 0) {
      MDCell& c = sc;
      B_V(a, c, h);
      cell_rates(c, rate[0]);               // B_R
      A_V(c, h);
      cell_rates(c, rate[1]);               // first A_R
      double z[3];
      normals3(a.seed, a.sysid, a.step, 0, kTagCell, z);
      const double c1 = exp(-a.gc * a.dt);
      const double amp = sqrt(a.ftm * a.kT * (1.0 - c1 * c1));
      if (c.mode == 0) c.pV = c1 * c.pV + amp * sqrt(c.M) * z[0];
      else if (c.mode == 2) {
        for (int d = 0; d < 3; ++d) c.pl[d] = c1 * c.pl[d] + amp * sqrt(c.Ml[d]) * z[d];
      } else {
        c.pA = c1 * c.pA + amp * sqrt(c.MA) * z[0];
        c.pL = c1 * c.pL + amp * sqrt(c.ML) * z[1];
      }
      cell_rates(c, rate[2]);               // second A_R
      A_V(c, h);
      cell_lengths(c);
      c.step = a.step;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (bx == 0 && lane < kCellWords)
      reinterpret_cast<uint64_t*>(a.cell_out)[lane] = reinterpret_cast<const uint64_t*>(&sc)[lane];
    if (lane < 9) {
      const int set = lane / 3, d = lane % 3;
      const double ra = rate[set][d];
      if (set == 0) { fac.eB[d] = exp(-ra * h); fac.fB[d] = expm1_over(-ra, h); }
      else if (set == 1) {
        fac.eA1[d] = exp(ra * h); fac.fA1[d] = expm1_over(ra, h); fac.iA1[d] = 1.0 / fac.fA1[d];
      } else {
        fac.eA2[d] = exp(ra * h); fac.fA2[d] = expm1_over(ra, h); fac.iA2[d] = 1.0 / fac.fA2[d];
      }
    }
  } else if (u < units) {
    // the noise of atom slot `wave` of unit u (a free atom has slot 0 only)
    int64_t i = -1;
    if (u < a.rig_count) i = a.rig_first + 3 * u + wave;
    else if (wave == 0) i = free_atom(a, u - a.rig_count);
    if (i >= 0) normals3(a.seed, a.sysid, a.step, (uint64_t)i, kTagNoise, zs[wave][lane]);
  }
  __syncthreads();
  if (wave != 0 || u >= units) return;
  const double c1 = exp(-a.gp * a.dt);
  if (rig) {
    const int64_t i0 = a.rig_first + 3 * u;
    const double im[3] = {1.0 / m[0], 1.0 / m[1], 1.0 / m[2]}, iM = 1.0 / (m[0] + m[1] + m[2]);
    const double ira = 1.0 / a.ra, i2rc = 1.0 / (2.0 * a.rc);
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int d = 0; d < 3; ++d)
        p[k][d] = p[k][d] * fac.eB[d] + a.ftm * F[k][d] * fac.fB[d];                         // B_R
    rigid_momenta(r, p, m, iM);
    bool ok = rigid_drift(a, r, p, m, im, iM, fac.eA1, fac.fA1, fac.iA1, ira, i2rc);         // A_R
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double amp = sqrt(a.ftm * a.kT * m[k] * (1.0 - c1 * c1));
#pragma unroll
      for (int d = 0; d < 3; ++d) p[k][d] = c1 * p[k][d] + amp * zs[k][lane][d];             // O
    }
    rigid_momenta(r, p, m, iM);
    ok = rigid_drift(a, r, p, m, im, iM, fac.eA2, fac.fA2, fac.iA2, ira, i2rc) && ok;        // A_R
    if (!ok) atomicOr(a.flags, 1);
    for (int k = 0; k < 3; ++k) {
      const int64_t i = i0 + k;
      a.x[i] = r[k][0]; a.y[i] = r[k][1]; a.z[i] = r[k][2];
      a.px[i] = p[k][0]; a.py[i] = p[k][1]; a.pz[i] = p[k][2];
    }
    return;
  }
  const int64_t i = free_atom(a, u - a.rig_count);
  const double im = 1.0 / m[0];
  const double amp = sqrt(a.ftm * a.kT * m[0] * (1.0 - c1 * c1));
  double* rr = r[0];
  double* pp = p[0];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    pp[d] = pp[d] * fac.eB[d] + a.ftm * F[0][d] * fac.fB[d];     // B_R
    rr[d] = rr[d] * fac.eA1[d] + pp[d] * im * fac.fA1[d];        // A_R
    pp[d] = c1 * pp[d] + amp * zs[0][lane][d];                   // O
    rr[d] = rr[d] * fac.eA2[d] + pp[d] * im * fac.fA2[d];        // A_R
  }
  a.x[i] = rr[0]; a.y[i] = rr[1]; a.z[i] = rr[2];
  a.px[i] = pp[0]; a.py[i] = pp[1]; a.pz[i] = pp[2];
}

__device__ __forceinline__ double wsum_md(double v) {
#pragma unroll
  for (int off = kMdThreads / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kMdThreads);
  return v;
}

// mode 0: closing half step (B_R, pressure, B_V); mode 1: pressure only
__device__ __forceinline__ void md_second_body(const MDArgs& a, int prime, int bx, int nbx) {
  __shared__ MDCell sc;
  __shared__ double sh[(kMdThreads + 63) / 64][12];
  __shared__ int sh_last;
  const double h = 0.5 * a.dt;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t u = (int64_t)bx * blockDim.x + threadIdx.x;
  // the unit's state is requested before the cell (independent loads)
  const bool rig = u < md_units(a) && u < a.rig_count;
  double r[3][3], p[3][3], F[3][3], m[3];
  if (rig) {
    const int64_t i0 = a.rig_first + 3 * u;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int64_t i = i0 + k;
      m[k] = a.mass[i];
      r[k][0] = a.x[i]; r[k][1] = a.y[i]; r[k][2] = a.z[i];
      p[k][0] = a.px[i]; p[k][1] = a.py[i]; p[k][2] = a.pz[i];
      F[k][0] = a.fx[i]; F[k][1] = a.fy[i]; F[k][2] = a.fz[i];
    }
  }
  // the cell, word by word; the virials (outputs of earlier launches, read
  // only by the block that closes the step) are requested now as well
  constexpr int kCellWords = sizeof(MDCell) / 8;
  static_assert(sizeof(MDCell) % 8 == 0 && kCellWords <= kMdThreads, "cell copied by one block");
  if (threadIdx.x < kCellWords)
    reinterpret_cast<uint64_t*>(&sc)[threadIdx.x] = reinterpret_cast<const uint64_t*>(a.cell_in)[threadIdx.x];
  double wv = 0.0;
  if (threadIdx.x < 6) {
    if (a.virial_k) wv += a.virial_k[threadIdx.x];
    if (a.virial_r) wv += a.virial_r[threadIdx.x];
  }
  __syncthreads();
  double rate[3];
  cell_rates(sc, rate);
  double k6[6] = {0, 0, 0, 0, 0, 0};   // kinetic tensor
  double c6[6] = {0, 0, 0, 0, 0, 0};   // molecular correction sum sym((r - R) F)
  if (rig) {
    const int64_t i0 = a.rig_first + 3 * u;
    if (!prime)
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int d = 0; d < 3; ++d)
          p[k][d] = p[k][d] * exp(-rate[d] * h) + a.ftm * F[k][d] * expm1_over(-rate[d], h);
    const double iM = 1.0 / (m[0] + m[1] + m[2]);
    rigid_momenta(r, p, m, iM);
    double P[3], R[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      P[d] = p[0][d] + p[1][d] + p[2][d];
      R[d] = (m[0] * r[0][d] + m[1] * r[1][d] + m[2] * r[2][d]) * iM;
    }
    k6[0] = P[0] * P[0] * iM; k6[1] = P[1] * P[1] * iM; k6[2] = P[2] * P[2] * iM;
    k6[3] = P[0] * P[1] * iM; k6[4] = P[0] * P[2] * iM; k6[5] = P[1] * P[2] * iM;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double x0 = r[k][0] - R[0], x1 = r[k][1] - R[1], x2 = r[k][2] - R[2];
      c6[0] += x0 * F[k][0]; c6[1] += x1 * F[k][1]; c6[2] += x2 * F[k][2];
      c6[3] += 0.5 * (x0 * F[k][1] + x1 * F[k][0]);
      c6[4] += 0.5 * (x0 * F[k][2] + x2 * F[k][0]);
      c6[5] += 0.5 * (x1 * F[k][2] + x2 * F[k][1]);
      const int64_t i = i0 + k;
      a.px[i] = p[k][0]; a.py[i] = p[k][1]; a.pz[i] = p[k][2];
    }
  } else if (u < md_units(a)) {
    const int64_t i = free_atom(a, u - a.rig_count);
    double p[3] = {a.px[i], a.py[i], a.pz[i]};
    if (!prime) {
      const double F[3] = {a.fx[i], a.fy[i], a.fz[i]};
#pragma unroll
      for (int d = 0; d < 3; ++d)
        p[d] = p[d] * exp(-rate[d] * h) + a.ftm * F[d] * expm1_over(-rate[d], h);
      a.px[i] = p[0]; a.py[i] = p[1]; a.pz[i] = p[2];
    }
    const double im = 1.0 / a.mass[i];
    k6[0] = p[0] * p[0] * im; k6[1] = p[1] * p[1] * im; k6[2] = p[2] * p[2] * im;
    k6[3] = p[0] * p[1] * im; k6[4] = p[0] * p[2] * im; k6[5] = p[1] * p[2] * im;
  }
  for (int k = 0; k < 6; ++k) {
    const double s = wsum_md(k6[k]);
    const double t = wsum_md(c6[k]);
    if (lane == 0) { sh[wave][k] = s; sh[wave][6 + k] = t; }
  }
  __syncthreads();
  if (threadIdx.x < 12) {
    double s = 0.0;
    for (int q = 0; q < (kMdThreads + 63) / 64; ++q) s += sh[q][threadIdx.x];
    __hip_atomic_store(&a.part[bx * 16 + threadIdx.x], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  // the last block of each group of kMdGroup blocks sums the group (one
  // block per thread, all loads in flight at once), the last group sums the
  // groups; both in a fixed order
  __shared__ double red[12][kMdThreads + 1];
  __shared__ double ksum[18];
  const int g = bx / kMdGroup, ng = (nbx + kMdGroup - 1) / kMdGroup;
  const int gsize = min(kMdGroup, nbx - g * kMdGroup);
  if (threadIdx.x == 0)
    sh_last = __hip_atomic_fetch_add(&a.cnt[g], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (unsigned)gsize - 1u;
  __syncthreads();
  if (!sh_last) return;
  static_assert(kMdGroup <= kMdThreads, "one group member per thread");
  {
    double pv[12];
#pragma unroll
    for (int k = 0; k < 12; ++k)
      pv[k] = (int)threadIdx.x < gsize ? __hip_atomic_load(&a.part[(g * kMdGroup + threadIdx.x) * 16 + k],
                                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0.0;
#pragma unroll
    for (int k = 0; k < 12; ++k) red[k][threadIdx.x] = pv[k];
  }
  __syncthreads();
  double* gp = a.part + (int64_t)nbx * 16;
  if (threadIdx.x < 12) {
    double s = 0.0;
    for (int j = 0; j < gsize; ++j) s += red[threadIdx.x][j];
    __hip_atomic_store(&gp[g * 16 + threadIdx.x], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (threadIdx.x == 0) __hip_atomic_store(&a.cnt[g], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0)
    sh_last = __hip_atomic_fetch_add(&a.cnt[ng], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (unsigned)ng - 1u;
  __syncthreads();
  if (!sh_last) return;
  {
    // thread t adds groups t, t + kMdThreads, ... in turn; then thread k adds
    // the threads' sums in order
    double pv[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int gi = threadIdx.x; gi < ng; gi += kMdThreads) {
#pragma unroll
      for (int k = 0; k < 12; ++k)
        pv[k] += __hip_atomic_load(&gp[gi * 16 + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) red[k][threadIdx.x] = pv[k];
  }
  __syncthreads();
  if (threadIdx.x < 12) {
    double s = 0.0;
    const int m = min(ng, kMdThreads);
    for (int j = 0; j < m; ++j) s += red[threadIdx.x][j];
    ksum[threadIdx.x] = s;
  }
  if (threadIdx.x < 6) ksum[12 + threadIdx.x] = wv;
  __syncthreads();
  if (threadIdx.x == 0) {
    MDCell& c = sc;
    const double iV = 1.0 / cell_volume(c);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      c.K[k] = ksum[k];
      c.C[k] = ksum[6 + k];
      c.P_ins[k] = (ksum[k] + a.ftm * (ksum[12 + k] - ksum[6 + k])) * iV;
    }
    if (!prime) B_V(a, c, h);
    __hip_atomic_store(&a.cnt[ng], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  if (threadIdx.x < kCellWords)
    reinterpret_cast<uint64_t*>(a.cell_out)[threadIdx.x] = reinterpret_cast<const uint64_t*>(&sc)[threadIdx.x];
}

__global__ void __launch_bounds__(kMdFirstThreads) k_md_first(MDArgs a) { md_first_body(a, blockIdx.x); }
__global__ void __launch_bounds__(kMdThreads) k_md_second(MDArgs a, int prime) {
  md_second_body(a, prime, blockIdx.x, gridDim.x);
}

hipError_t launch_md_first(const MDArgs& a, hipStream_t s) {
  const unsigned blocks = (unsigned)md_blocks(md_units(a));
  hipLaunchKernelGGL(k_md_first, dim3(blocks), dim3(kMdFirstThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_md_second(const MDArgs& a, int prime, hipStream_t s) {
  const unsigned blocks = (unsigned)md_blocks(md_units(a));
  hipLaunchKernelGGL(k_md_second, dim3(blocks), dim3(kMdThreads), 0, s, a, prime);
  return hipGetLastError();
}

// many systems per launch (block b -> system s with bstart[s] <= b < bstart[s+1])
__device__ __forceinline__ int find_sys_m(const int* bstart, int nsys, int b) {
  int lo = 0, hi = nsys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bstart[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void __launch_bounds__(kMdFirstThreads) k_md_first_m(const MDArgs* tab, const int* bstart, int nsys) {
  __shared__ MDArgs sa;
  const int sys = find_sys_m(bstart, nsys, blockIdx.x);
  if (threadIdx.x == 0) sa = tab[sys];
  __syncthreads();
  md_first_body(sa, blockIdx.x - bstart[sys]);
}

__global__ void __launch_bounds__(kMdThreads) k_md_second_m(const MDArgs* tab, const int* bstart, int nsys,
                                                     int prime) {
  __shared__ MDArgs sa;
  const int sys = find_sys_m(bstart, nsys, blockIdx.x);
  if (threadIdx.x == 0) sa = tab[sys];
  __syncthreads();
  md_second_body(sa, prime, blockIdx.x - bstart[sys], bstart[sys + 1] - bstart[sys]);
}

hipError_t launch_md_first_multi(const MDArgs* d_tab, const int* d_bstart, int nsys, int total,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_md_first_m, dim3(total), dim3(kMdFirstThreads), 0, s, d_tab, d_bstart, nsys);
  return hipGetLastError();
}

hipError_t launch_md_second_multi(const MDArgs* d_tab, const int* d_bstart, int nsys, int total,
                                  int prime, hipStream_t s) {
  hipLaunchKernelGGL(k_md_second_m, dim3(total), dim3(kMdThreads), 0, s, d_tab, d_bstart, nsys, prime);
  return hipGetLastError();
}

}  // namespace rbe
