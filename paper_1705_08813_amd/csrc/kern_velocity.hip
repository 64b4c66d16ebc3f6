// Enriched DG velocity residual (arXiv 1705.08813, Sec. 3.1 and 4.2):
// local Lax-Friedrichs convective term + interior-penalty viscous term on the
// space u = u_bar + psi sum_B N^l_B u~_B (enrichment in the wall-adjacent
// layer; weights of degree l = 0, one coefficient per component, or l = 1,
// the eight trilinear vertex functions of the cell, eq. enrichment).
//
// One workgroup per cell.  The cell's nodal values are staged in LDS; values
// and gradients at the Gauss points come from sum-factorized sweeps (basis
// interpolation, then collocation derivatives through the Gauss points); the
// pointwise flux is integrated back with the transposed sweeps.  Faces are
// handled element by element: each cell evaluates its own and its
// neighbour's traces on each of its six faces and integrates the numerical
// flux against its own test functions, so every output has one writer and no
// atomics are needed.  Enriched cells run a separate instantiation whose
// wall-normal rule has NQY points and which reads the precomputed psi and
// grad psi tables.
#include <cstring>

#include "kern_common.h"

namespace dgwm {

namespace {

template <typename T, int NP, int NQ, int NQY>
struct VelShape {
  static constexpr int NP2 = NP * NP, NP3 = NP * NP * NP;
  static constexpr int NPTS = NQ * NQY * NQ;
  static constexpr int FMAX = (NQ * NQY > NQ * NQ) ? NQ * NQY : NQ * NQ;
  static constexpr int Q1MAX = NQY > NQ ? NQY : NQ;
  static constexpr int NL = 6 * 3 * 2 * NP2;            // neighbour layers [face][c][val|d_n][NP2]
  static constexpr int LAYO = 2 * 3 * 2 * NP2;          // own layers of the two faces of one direction
  static constexpr int A1 = 2 * 2 * 7 * Q1MAX * NP;     // t1-swept traces [s][side][field][q1][i2]
  static constexpr int FL = 2 * 8 * FMAX;               // fluxes [s][field][pt]
  static constexpr int B1 = 2 * 3 * 3 * Q1MAX * NP;     // t2-transposed tests [s][c][3][q1][i2]
  static constexpr int TRC = 2 * 2 * 8 * FMAX;          // traces [s][side][field][pt]
  static constexpr int FACE0 = NL + LAYO + A1 + TRC;
  static constexpr int FACE = FACE0 > NL + LAYO + A1 + FL + B1 ? FACE0 : NL + LAYO + A1 + FL + B1;
  // curved cells: 12 trace fields per side and reference-gradient tests
  static constexpr int A1C = 2 * 2 * 3 * 3 * Q1MAX * NP;
  static constexpr int FLC = 2 * 12 * FMAX;
  static constexpr int FACEC = NL + LAYO + A1C + FLC + B1;
  static constexpr int VOL = 12 * NPTS;
  static constexpr int BIG0 = VOL > FACE ? VOL : FACE;
  static constexpr int BIG = BIG0 > FACEC ? BIG0 : FACEC;
};

// Node index of the point at position l along direction D on the line
// (a, b) of the two tangential directions (t1 < t2):  base + l * stride.
template <int NP>
__device__ __forceinline__ void line_of(int D, int a, int b, int& base, int& stride) {
  if (D == 0) {
    base = NP * (a + NP * b);
    stride = 1;
  } else if (D == 1) {
    base = a + NP * NP * b;
    stride = NP;
  } else {
    base = a + NP * b;
    stride = NP * NP;
  }
}

// Neighbour of the current cell across face (D, S).
// Degree-1 enrichment weights (Sec. 3.1, eq. enrichment with l = 1): the
// trilinear vertex functions N_B = prod_d (b_d ? xi_d : 1 - xi_d) of the
// reference point xi, B = bx + 2 (by + 2 bz), and their physical derivatives
// on an affine cell (ih: reciprocal cell sizes).
template <typename T>
__device__ __forceinline__ void vertex_fns(const T xi[3], const T ih[3], T n[8], T dn[3][8]) {
  const T v[3][2] = {{T(1) - xi[0], xi[0]}, {T(1) - xi[1], xi[1]}, {T(1) - xi[2], xi[2]}};
#pragma unroll
  for (int B = 0; B < 8; ++B) {
    const int bx = B & 1, by = (B >> 1) & 1, bz = B >> 2;
    n[B] = v[0][bx] * v[1][by] * v[2][bz];
    dn[0][B] = (bx ? ih[0] : -ih[0]) * v[1][by] * v[2][bz];
    dn[1][B] = (by ? ih[1] : -ih[1]) * v[0][bx] * v[2][bz];
    dn[2][B] = (bz ? ih[2] : -ih[2]) * v[0][bx] * v[1][by];
  }
}

// The weight field L_c = sum_B N_B ut[c][B] and its gradient dL[c][d].
template <typename T>
__device__ __forceinline__ void vertex_weight(const T* ut, const T n[8], const T dn[3][8], T L[3], T dL[3][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T a = 0, g0 = 0, g1 = 0, g2 = 0;
#pragma unroll
    for (int B = 0; B < 8; ++B) {
      const T w = ut[c * 8 + B];
      a += n[B] * w;
      g0 += dn[0][B] * w;
      g1 += dn[1][B] * w;
      g2 += dn[2][B] * w;
    }
    L[c] = a;
    dL[c][0] = g0;
    dL[c][1] = g1;
    dL[c][2] = g2;
  }
}

struct FaceNb {
  int64_t enb;     // neighbour cell (valid unless wall)
  int64_t enr_nb;  // its enriched index or -1
  bool wall;
  int nidx1;       // neighbour's ey (for its height)
};

// (cell counts stay below 2^31, checked at set-up)
__device__ __forceinline__ FaceNb face_nb(const MeshDev& M, int ex, int ey, int ez, int D, int S) {
  const int nmax = D == 0 ? M.nx : (D == 1 ? M.ny : M.nz);
  int j = (D == 0 ? ex : (D == 1 ? ey : ez)) + (S ? 1 : -1);
  FaceNb f;
  f.wall = false;
  if (j < 0 || j >= nmax) {
    if (D == 1 && !M.fully_periodic) f.wall = true;
    j += j < 0 ? nmax : -nmax;
  }
  const int n0 = D == 0 ? j : ex, n1 = D == 1 ? j : ey, n2 = D == 2 ? j : ez;
  f.enb = n0 + M.nx * (n1 + M.ny * n2);
  f.enr_nb = f.wall ? -1 : enr_index(M, n0, n1, n2);
  f.nidx1 = n1;
  return f;
}

// Neighbour face layers of all six faces: value and normal derivative of each
// component on the neighbour's node layer at the shared face.  The lines of
// neighbour nodes are fetched into registers when the cell starts (nb_fetch),
// so their latency overlaps the volume term, and reduced to value and
// derivative into LDS right before the face phases (nb_store).
template <typename T, int NP>
struct NbLines {
  static constexpr int NP2 = NP * NP, N = 6 * 3 * NP2, ITEMS = (N + 255) / 256;
  T x[ITEMS][NP];
  T nut;  // enrichment coefficient of a neighbour (threads 0..18 LE - 1: face f = tid / (3 LE),
          // then [component][enrichment node])
};

template <typename T, int NP, int LE = 1>
__device__ __forceinline__ void nb_fetch(const MeshDev& M, const T* __restrict__ u, int ex, int ey, int ez,
                                         NbLines<T, NP>& L) {
  using NL = NbLines<T, NP>;
  constexpr int NP2 = NL::NP2, NP3 = NP * NP * NP;
#pragma unroll
  for (int it = 0; it < NL::ITEMS; ++it) {
    const int t = threadIdx.x + 256 * it;
#pragma unroll
    for (int l = 0; l < NP; ++l) L.x[it][l] = 0;
    if (t < NL::N) {
      const int f = t / (3 * NP2), rem = t - f * 3 * NP2;
      const int c = rem / NP2, k = rem - c * NP2;
      const FaceNb nb = face_nb(M, ex, ey, ez, f >> 1, f & 1);
      if (!nb.wall) {
        int base, stride;
        line_of<NP>(f >> 1, k % NP, k / NP, base, stride);
        const T* src = u + (nb.enb * 3 + c) * NP3 + base;
#pragma unroll
        for (int l = 0; l < NP; ++l) L.x[it][l] = src[l * stride];
      }
    }
  }
  L.nut = 0;
  if (threadIdx.x < 18 * LE) {
    const int f = threadIdx.x / (3 * LE), k = threadIdx.x % (3 * LE);
    const FaceNb nb = face_nb(M, ex, ey, ez, f >> 1, f & 1);
    if (nb.enr_nb >= 0) L.nut = u[M.enr_off + nb.enr_nb * 3 * LE + k];
  }
}

// ihn: reciprocal size along the face normal of the neighbours across the
// faces y = 0 and y = 1 of the cell (x and z sizes are uniform)
template <typename T, int NP, int NQ, bool REF, int LE = 1>
__device__ __forceinline__ void nb_store(const MeshDev& M, const NbLines<T, NP>& L, T* s_nl, T* s_nut, int ex, int ey,
                                         int ez, T ihx, T ihz, T ihy0, T ihy1) {
  using NL = NbLines<T, NP>;
  constexpr int NP2 = NL::NP2;
  constexpr auto& tb = ct::tab<NP, NQ>;
#pragma unroll
  for (int it = 0; it < NL::ITEMS; ++it) {
    const int t = threadIdx.x + 256 * it;
    if (t < NL::N) {
      const int f = t / (3 * NP2), rem = t - f * 3 * NP2;
      const int c = rem / NP2, k = rem - c * NP2;
      const int D = f >> 1, S = f & 1;
      T val = 0, der = 0;
      const FaceNb nb = face_nb(M, ex, ey, ez, D, S);
      if (!nb.wall) {
        // the neighbour's face is at xi_D = 1 - S (both sums, one select:
        // a per-lane choice of coefficients would cost a select per term)
        T d0 = 0, d1 = 0;
#pragma unroll
        for (int l = 0; l < NP; ++l) {
          d0 += T(tb.nd0[l]) * L.x[it][l];
          d1 += T(tb.nd1[l]) * L.x[it][l];
        }
        der = S ? d0 : d1;
        val = S ? L.x[it][0] : L.x[it][NP - 1];
        if (!REF)  // affine cells: physical normal derivative
          der *= D == 0 ? ihx : (D == 1 ? (S ? ihy1 : ihy0) : ihz);
      }
      s_nl[((f * 3 + c) * 2 + 0) * NP2 + k] = val;
      s_nl[((f * 3 + c) * 2 + 1) * NP2 + k] = der;
    }
  }
  if (threadIdx.x < 18 * LE) s_nut[threadIdx.x] = L.nut;
}

// 1-D tables used by the face phases, staged in LDS in the working precision
// (their indices vary across lanes there): S, S' of the wall-parallel rule and
// of the cell's wall-normal rule, both weight vectors, N'(0) and N'(1).
template <int NP, int NQ, int NQY>
struct FaceTab {
  static constexpr int Sq = 0, Sdq = Sq + NQ * NP, Sy = Sdq + NQ * NP, Sdy = Sy + NQY * NP;
  static constexpr int wq = Sdy + NQY * NP, wy = wq + NQ, nd0 = wy + NQY, nd1 = nd0 + NP, size = nd1 + NP;
};

template <typename T, int NP, int NQ, int NQY, bool ENR>
__device__ __forceinline__ void load_face_tab(const double* tab, T* s_tab) {
  using TL = FaceTab<NP, NQ, NQY>;
  constexpr TabLayout L = tab_layout(NP, NQ, NQY);
  for (int i = threadIdx.x; i < TL::size; i += blockDim.x) {
    double v;
    if (i < TL::Sdq) v = tab[L.S + i];
    else if (i < TL::Sy) v = tab[L.Sd + i - TL::Sdq];
    else if (i < TL::Sdy) v = tab[(ENR ? L.Sy : L.S) + i - TL::Sy];
    else if (i < TL::wq) v = tab[(ENR ? L.Sdy : L.Sd) + i - TL::Sdy];
    else if (i < TL::wy) v = tab[L.w + i - TL::wq];
    else if (i < TL::nd0) v = tab[(ENR ? L.wy : L.w) + i - TL::wy];
    else if (i < TL::nd1) v = tab[L.nd0 + i - TL::nd0];
    else v = tab[L.nd1 + i - TL::nd1];
    s_tab[i] = T(v);
  }
}

// One face point of the multiscale viscous operator (Sec. 4.2, eq.
// viscous_multiscale; -F^nu_e, adjoint sign -1) in the general face phase.
// tr holds the polynomial traces of both sides (own: tr[0]; neighbour:
// tr[1], unset on a wall) in the layout of vel_faces_dir; the enrichment
// parts u~ = psi ut come from the psi tables.  Face classes: an enriched
// cell's face is "inner" when its other side is enriched or a wall (mirror
// side), "interface" otherwise; a cell without enrichment sees "regular" or
// "interface" faces, which take the same form with the jump of the full
// velocity.  Writes the weighted value flux, F_g[c][D], F_g[D][T1] and
// F_g[D][T2] in the vel_faces_dir layout and adds the face terms of the
// enrichment test rows to rt.  With degree-1 weights (LE = 8) u~ = psi sum_B
// N_B ut_B and the test functions are psi N_B e_c; (x1, x2) are the point's
// tangential reference coordinates, ih the cell's reciprocal sizes and ihn
// the neighbour's along D.
template <typename T, bool ENR, int D, int T1, int T2, int LE = 1>
__device__ __forceinline__ void vel_ms_face_point(const MeshDev& M, const T (&tr)[2][8], int s, int pt, int FP,
                                                  bool wall, int64_t enr_nb, int64_t enr, const T* s_ut,
                                                  const T* s_nut, T wf, T tau, T* fo, T* rt, T x1 = T(0),
                                                  T x2 = T(0), const T* ih = nullptr, T ihn = T(0)) {
  const T nu = T(M.nu);
  const T sg = s ? T(1) : T(-1);
  const int f = 2 * D + s, fn = 2 * D + (1 - s);
  // normal column of the symmetric polynomial gradient, (grad u + grad u^T)_{cD}
  auto sym = [&](const T* t, int c) {
    return c == D ? T(2) * t[3 + D] : (c == T1 ? t[3 + c] + t[6] : t[3 + c] + t[7]);
  };
  T ubm[3], ubp[3], sbm[3], sbp[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    ubm[c] = tr[0][c];
    sbm[c] = sym(tr[0], c);
    ubp[c] = wall ? -ubm[c] : tr[1][c];
    sbp[c] = wall ? sbm[c] : sym(tr[1], c);
  }
  // enrichment parts: u~ = psi ut, (grad u~ + grad u~^T)_{cD} = ut_c dD psi + ut_D dc psi
  T utm[3] = {0, 0, 0}, stm[3] = {0, 0, 0}, utp[3] = {0, 0, 0}, stp[3] = {0, 0, 0};
  T psim = 0, gpsim[3] = {0, 0, 0}, num = 0, nup = 0;
  T nB[LE], dB[3][LE];  // degree-1 weights: own vertex functions at the point
  if (ENR) {
    const double* ps = M.psi + ((size_t)enr * M.psi_pts + M.psi_off[1 + f] + pt) * 4;
    psim = T(ps[0]);
    gpsim[0] = T(ps[1]);
    gpsim[1] = T(ps[2]);
    gpsim[2] = T(ps[3]);
    num = T(M.nut[(size_t)enr * M.psi_pts + M.psi_off[1 + f] + pt]);
    if constexpr (LE == 1) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        utm[c] = psim * s_ut[c];
        stm[c] = s_ut[c] * gpsim[D] + s_ut[D] * gpsim[c];
      }
    } else {
      T xi[3], L[3], dL[3][3];
      xi[D] = T(s);
      xi[T1] = x1;
      xi[T2] = x2;
      vertex_fns(xi, ih, nB, dB);
      vertex_weight(s_ut, nB, dB, L, dL);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        utm[c] = psim * L[c];
        stm[c] = (L[c] * gpsim[D] + psim * dL[c][D]) + (L[D] * gpsim[c] + psim * dL[D][c]);
      }
    }
  }
  const bool nb_enr = !wall && enr_nb >= 0;
  if (wall) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      utp[c] = -utm[c];
      stp[c] = stm[c];
    }
    nup = num;
  } else if (nb_enr) {
    const size_t q = (size_t)enr_nb * M.psi_pts + M.psi_off[1 + fn] + pt;
    const double* ps = M.psi + q * 4;
    const T psip = T(ps[0]);
    const T gpp[3] = {T(ps[1]), T(ps[2]), T(ps[3])};
    const T* ut = s_nut + f * 3 * LE;
    nup = T(M.nut[q]);
    if constexpr (LE == 1) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        utp[c] = psip * ut[c];
        stp[c] = ut[c] * gpp[D] + ut[D] * gpp[c];
      }
    } else {
      T xin[3], ihv[3] = {ih[0], ih[1], ih[2]}, nn[8], dn[3][8], L[3], dL[3][3];
      xin[D] = T(1 - s);
      xin[T1] = x1;
      xin[T2] = x2;
      ihv[D] = ihn;
      vertex_fns(xin, ihv, nn, dn);
      vertex_weight(ut, nn, dn, L, dL);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        utp[c] = psip * L[c];
        stp[c] = (L[c] * gpp[D] + psip * dL[c][D]) + (L[D] * gpp[c] + psip * dL[D][c]);
      }
    }
  }
  const bool inner = ENR && (wall || nb_enr);
  // harmonic weights of the averages with nu + nu_t (eq. harmweights)
  const T den = T(2) * nu + num + nup;
  const T wm = inner ? (nu + nup) / den : T(0.5), wp = inner ? (nu + num) / den : T(0.5);
  T jb[3], ju[3], Eb[3], Et[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    jb[c] = ubm[c] - ubp[c];
    ju[c] = (ubm[c] + utm[c]) - (ubp[c] + utp[c]);
    Eb[c] = T(0.5) * nu * sg * (sbm[c] + sbp[c]);
    Et[c] = inner ? sg * (wm * (nu + num) * stm[c] + wp * (nu + nup) * stp[c]) : T(0);
  }
  const T* J = inner ? jb : ju;
  const T hn = T(0.5) * nu * sg;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T fv = -Eb[c] - Et[c] + tau * nu * ju[c];
    fo[c * FP] = wf * fv;
    fo[(3 + c) * FP] = wf * (c == D ? T(2) : T(1)) * hn * J[c];
  }
  fo[6 * FP] = wf * hn * J[T1];
  fo[7 * FP] = wf * hn * J[T2];
  if constexpr (ENR && LE == 1) {
    const T gn = sg * gpsim[D];
    const T jg = ju[0] * gpsim[0] + ju[1] * gpsim[1] + ju[2] * gpsim[2];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T val = inner ? psim * (-Et[c] + tau * nu * ju[c]) + wm * (nu + num) * (ju[c] * gn + (c == D ? jg * sg : T(0)))
                          : psim * (-Eb[c] + tau * nu * ju[c]);
      rt[c] += wf * val;
    }
  }
  if constexpr (ENR && LE == 8) {
    // test functions phi e_c, phi = psi N_B, grad phi = N_B grad psi + psi grad N_B
#pragma unroll
    for (int B = 0; B < 8; ++B) {
      const T phi = psim * nB[B];
      T gp[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) gp[d] = nB[B] * gpsim[d] + psim * dB[d][B];
      const T gn = sg * gp[D];
      const T jg = ju[0] * gp[0] + ju[1] * gp[1] + ju[2] * gp[2];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T val = inner ? phi * (-Et[c] + tau * nu * ju[c]) + wm * (nu + num) * (ju[c] * gn + (c == D ? jg * sg : T(0)))
                            : phi * (-Eb[c] + tau * nu * ju[c]);
        rt[c * 8 + B] += wf * val;
      }
    }
  }
}

// Both faces of direction D: traces on both sides at the face Gauss points
// (factorized 2-D interpolation of the node layers), numerical flux, and
// integration against the cell's own test functions (transposed sweeps).
//
// With the normal n = +-e_D, the fluxes use only 8 trace fields per side:
// u_c, d_D u_c (c = 0..2), and the tangential derivatives d_T1 u_D, d_T2 u_D
// ({{2 nu eps(u)}} n needs (grad u + grad u^T) e_D), and the adjoint term
// -theta nu sym(j (x) n) tests only d_D phi_c and d_T phi_D.
//
// Every 1-D contraction runs as a thread-owned line with the table entries
// as literals of the unrolled code (one LDS read per input, none per
// coefficient); phases are separated by workgroup barriers.
template <typename T, int NP, int NQ, int NQY, bool ENR, int D, bool MS = false, int LE = 1>
__device__ __forceinline__ void vel_faces_dir(const MeshDev& M, const T* s_u, const T* s_nl, const T* s_nut, T* s_r,
                                              T* s_face, const T* s_ut, int ex, int ey, int ez, int64_t enr, T hx,
                                              T hy, T hz, T ihx, T ihy, T ihz, T* rt) {
  static_assert(LE == 1 || LE == 8, "enrichment weights of degree 0 or 1");
  using Sh = VelShape<T, NP, NQ, NQY>;
  constexpr int T1 = D == 0 ? 1 : 0;
  constexpr int T2 = D == 2 ? 1 : 2;
  constexpr int Q1 = T1 == 1 ? NQY : NQ;
  constexpr int Q2 = T2 == 1 ? NQY : NQ;
  constexpr int FP = Q1 * Q2;
  constexpr int NP2 = Sh::NP2, NP3 = Sh::NP3;
  constexpr auto& tb1 = ct::tab<NP, Q1>;
  constexpr auto& tb2 = ct::tab<NP, Q2>;
  constexpr auto& tbn = ct::tab<NP, NQ>;  // nd0, nd1 do not depend on the rule
  const int tid = threadIdx.x;
  constexpr int nt = 256;  // workgroup size of every velocity launch

  // LDS regions (see VelShape::FACE): X = own layers, later fluxes and line
  // results; Y = t1-swept traces; Z = traces, later t2-transposed tests
  T* lay = s_face;                     // [s][c][val|d_n][NP2]
  T* A1 = lay + Sh::LAYO;              // [s][side][field 0..6][q1][i2]
  T* TR = A1 + Sh::A1;                 // [s][side][field 0..7][pt]
  T* FL = s_face;                      // [s][field 0..7][pt]
  T* B1 = TR;                          // [s][test 0..6][q1][i2]
  T* RB = s_face;                      // [s][c][value|normal][NP2]

  const T hown[3] = {hx, hy, hz}, ihown[3] = {ihx, ihy, ihz};
  const T ht1 = hown[T1], ht2 = hown[T2];
  const T ihd = ihown[D], iht1 = ihown[T1], iht2 = ihown[T2];
  const FaceNb nb0 = face_nb(M, ex, ey, ez, D, 0), nb1 = face_nb(M, ex, ey, ez, D, 1);
  // tau = pen max(1/h-, 1/h+)
  auto tau_of = [&](const FaceNb& nb) {
    if (nb.wall) return T(M.pen * M.wall_mult) * ihd;
    if (D != 1) return T(M.pen) * ihd;
    const T ihn = T(M.ihy[nb.nidx1]);
    return T(M.pen) * (ihd > ihn ? ihd : ihn);
  };
  const T tau0 = tau_of(nb0), tau1 = tau_of(nb1);
  const bool wall0 = nb0.wall, wall1 = nb1.wall;
  const int64_t enrn0 = nb0.enr_nb, enrn1 = nb1.enr_nb;
  // neighbours' reciprocal sizes along D (degree-1 weights of an enriched neighbour)
  const T ihn0 = D == 1 ? T(M.ihy[nb0.nidx1]) : ihd, ihn1 = D == 1 ? T(M.ihy[nb1.nidx1]) : ihd;

  // psi and grad psi at this thread's point of the flux phase (C2 mapping),
  // of the own side (enriched cells) and of an enriched neighbour's side,
  // loaded here so that their latency overlaps the trace phases
  T pfo[4] = {0, 0, 0, 0}, pfn[4] = {0, 0, 0, 0};
  if constexpr (!MS) {
    const int q1 = tid & 7, q2 = (tid >> 3) & 7, s = tid >> 6;
    if (tid < 2 * 64 && q1 < Q1 && q2 < Q2) {
      const int pt = q1 + Q1 * q2;
      if (ENR) {
        const double* ps = M.psi + ((size_t)enr * M.psi_pts + M.psi_off[1 + 2 * D + s] + pt) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) pfo[j] = T(ps[j]);
      }
      const int64_t en = s ? enrn1 : enrn0;
      if (!(s ? wall1 : wall0) && en >= 0) {
        const double* ps = M.psi + ((size_t)en * M.psi_pts + M.psi_off[1 + 2 * D + (1 - s)] + pt) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) pfn[j] = T(ps[j]);
      }
    }
  }

  // Phase A: own node layers of both faces (value, d/dx_D), one line each
  for (int t = tid; t < 3 * NP2; t += nt) {
    const int c = t / NP2, k = t - c * NP2;
    int base, stride;
    line_of<NP>(D, k % NP, k / NP, base, stride);
    const T* src = s_u + c * NP3 + base;
    T x[NP];
#pragma unroll
    for (int l = 0; l < NP; ++l) x[l] = src[l * stride];
    T d0 = 0, d1 = 0;
#pragma unroll
    for (int l = 0; l < NP; ++l) {
      d0 += T(tbn.nd0[l]) * x[l];
      d1 += T(tbn.nd1[l]) * x[l];
    }
    lay[((0 * 3 + c) * 2 + 0) * NP2 + k] = x[0];
    lay[((0 * 3 + c) * 2 + 1) * NP2 + k] = d0 * ihd;
    lay[((1 * 3 + c) * 2 + 0) * NP2 + k] = x[NP - 1];
    lay[((1 * 3 + c) * 2 + 1) * NP2 + k] = d1 * ihd;
  }
  __syncthreads();

  // Phase B1: lines along t1 (node i1 -> Gauss q1).  Fields: 0-2 value of
  // u_c, 3-5 normal derivative of u_c, 6 t1-derivative of u_D.
  // Thread t takes line i2 = t & 7 of side (t >> 3) & 1, face (t >> 4) & 1,
  // field t >> 5: two fields per wavefront, so the derivative field 6 has
  // wavefront 3 to itself and no wavefront runs both branches; the index
  // decomposition is shifts and masks (NP <= 8).
  static_assert(NP <= 8 && Q1 <= 8 && Q2 <= 8, "face phases index lines and points in 3 bits");
  {
    const int t = tid;
    const int i2 = t & 7, side = (t >> 3) & 1, s = (t >> 4) & 1, f = t >> 5;
    if (f < 7 && i2 < NP && !(side == 1 && (s ? wall1 : wall0))) {
    const int c = f < 3 ? f : (f < 6 ? f - 3 : D);
    const int fld = (f >= 3 && f < 6) ? 1 : 0;
    const T* lv = (side == 0 ? lay + ((s * 3 + c) * 2) * NP2 : s_nl + (((2 * D + s) * 3 + c) * 2) * NP2) +
                  fld * NP2 + NP * i2;
    T x[NP];
#pragma unroll
    for (int i1 = 0; i1 < NP; ++i1) x[i1] = lv[i1];
    T* o = A1 + (((s * 2 + side) * 7 + f) * Q1) * NP + i2;
    if (f == 6) {
#pragma unroll
      for (int q1 = 0; q1 < Q1; ++q1) {
        T acc = 0;
#pragma unroll
        for (int i1 = 0; i1 < NP; ++i1) acc += T(tb1.Sd[q1][i1]) * x[i1];
        o[q1 * NP] = acc * iht1;
      }
    } else {
#pragma unroll
      for (int q1 = 0; q1 < Q1; ++q1) {
        T acc = 0;
#pragma unroll
        for (int i1 = 0; i1 < NP; ++i1) acc += T(tb1.S[q1][i1]) * x[i1];
        o[q1 * NP] = acc;
      }
    }
    }
  }
  __syncthreads();

  // Phase C1: lines along t2 (node i2 -> Gauss q2), giving the 8 trace
  // fields of each side; field 7 = d_T2 u_D from the value of u_D.
  // Thread t takes line q1 = t & 7 of side (t >> 3) & 1, face (t >> 4) & 1,
  // field t >> 5 (so only wavefront 3, fields 6 and 7, runs both branches).
  {
    const int t = tid;
    const int q1 = t & 7, side = (t >> 3) & 1, s = (t >> 4) & 1, fo = t >> 5;
    if (q1 < Q1 && !(side == 1 && (s ? wall1 : wall0))) {
    const int fin = fo < 7 ? fo : D;
    const T* a = A1 + (((s * 2 + side) * 7 + fin) * Q1 + q1) * NP;
    T x[NP];
#pragma unroll
    for (int i2 = 0; i2 < NP; ++i2) x[i2] = a[i2];
    T* o = TR + ((s * 2 + side) * 8 + fo) * FP + q1;
    if (fo == 7) {
#pragma unroll
      for (int q2 = 0; q2 < Q2; ++q2) {
        T acc = 0;
#pragma unroll
        for (int i2 = 0; i2 < NP; ++i2) acc += T(tb2.Sd[q2][i2]) * x[i2];
        o[q2 * Q1] = acc * iht2;
      }
    } else {
#pragma unroll
      for (int q2 = 0; q2 < Q2; ++q2) {
        T acc = 0;
#pragma unroll
        for (int i2 = 0; i2 < NP; ++i2) acc += T(tb2.S[q2][i2]) * x[i2];
        o[q2 * Q1] = acc;
      }
    }
    }
  }
  __syncthreads();

  // Phase C2: numerical flux at each face point (thread t: q1 = t & 7,
  // q2 = (t >> 3) & 7, face t >> 6; one pass over the first 128 threads)
  const T nu = T(M.nu), theta = T(M.theta);
  for (int t = tid; t < 2 * 64; t += nt) {
    const int q1 = t & 7, q2 = (t >> 3) & 7, s = t >> 6;
    if (q1 >= Q1 || q2 >= Q2) continue;
    const int pt = q1 + Q1 * q2;
    const T sg = s ? T(1) : T(-1);
    const bool wall = s ? wall1 : wall0;
    const int64_t enr_nb = s ? enrn1 : enrn0;
    // tr[side][0..2] u_c, [3..5] d_D u_c, [6] d_T1 u_D, [7] d_T2 u_D
    T tr[2][8];
#pragma unroll
    for (int f = 0; f < 8; ++f) tr[0][f] = TR[((s * 2 + 0) * 8 + f) * FP + pt];
    if (!wall) {
#pragma unroll
      for (int f = 0; f < 8; ++f) tr[1][f] = TR[((s * 2 + 1) * 8 + f) * FP + pt];
    }
    if constexpr (MS) {
      vel_ms_face_point<T, ENR, D, T1, T2, LE>(M, tr, s, pt, FP, wall, enr_nb, enr, s_ut, s_nut,
                                               T(tb1.w[q1]) * T(tb2.w[q2]) * ht1 * ht2, s ? tau1 : tau0,
                                               FL + s * 8 * FP + pt, rt, T(tb1.g[q1]), T(tb2.g[q2]), ihown,
                                               s ? ihn1 : ihn0);
      continue;
    }
    T psim = 0, gpsim[3] = {0, 0, 0};
    // degree-1 weights: vertex functions at the face point (own cell, xi_D = s)
    T nB[LE], dB[3][LE];
    if (ENR) {
      psim = pfo[0];
      gpsim[0] = pfo[1];
      gpsim[1] = pfo[2];
      gpsim[2] = pfo[3];
      if constexpr (LE == 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          tr[0][c] += psim * s_ut[c];
          tr[0][3 + c] += s_ut[c] * gpsim[D];
        }
        tr[0][6] += s_ut[D] * gpsim[T1];
        tr[0][7] += s_ut[D] * gpsim[T2];
      } else {
        // u~_c = psi L_c:  d_k u~_c = L_c d_k psi + psi d_k L_c
        T xi[3], L[3], dL[3][3];
        xi[D] = T(s);
        xi[T1] = T(tb1.g[q1]);
        xi[T2] = T(tb2.g[q2]);
        vertex_fns(xi, ihown, nB, dB);
        vertex_weight(s_ut, nB, dB, L, dL);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          tr[0][c] += psim * L[c];
          tr[0][3 + c] += L[c] * gpsim[D] + psim * dL[c][D];
        }
        tr[0][6] += L[D] * gpsim[T1] + psim * dL[D][T1];
        tr[0][7] += L[D] * gpsim[T2] + psim * dL[D][T2];
      }
    }
    if (wall) {
#pragma unroll
      for (int f = 0; f < 8; ++f) tr[1][f] = (f < 3) ? -tr[0][f] : tr[0][f];
    } else if (enr_nb >= 0) {
      const T psip = pfn[0];
      const T gpp[3] = {pfn[1], pfn[2], pfn[3]};
      const T* ut = s_nut + (2 * D + s) * 3 * LE;
      if constexpr (LE == 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          tr[1][c] += psip * ut[c];
          tr[1][3 + c] += ut[c] * gpp[D];
        }
        tr[1][6] += ut[D] * gpp[T1];
        tr[1][7] += ut[D] * gpp[T2];
      } else {
        // the neighbour's vertex functions at the same point (its xi_D = 1 - s)
        T xin[3], ihn[3] = {ihown[0], ihown[1], ihown[2]}, nn[8], dn[3][8], L[3], dL[3][3];
        xin[D] = T(1 - s);
        xin[T1] = T(tb1.g[q1]);
        xin[T2] = T(tb2.g[q2]);
        ihn[D] = s ? ihn1 : ihn0;
        vertex_fns(xin, ihn, nn, dn);
        vertex_weight(ut, nn, dn, L, dL);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          tr[1][c] += psip * L[c];
          tr[1][3 + c] += L[c] * gpp[D] + psip * dL[c][D];
        }
        tr[1][6] += L[D] * gpp[T1] + psip * dL[D][T1];
        tr[1][7] += L[D] * gpp[T2] + psip * dL[D][T2];
      }
    }
    // n = sg e_D
    const T unm = sg * tr[0][D], unp = sg * tr[1][D];
    const T am = unm < 0 ? -unm : unm, ap = unp < 0 ? -unp : unp;
    const T lam = T(2) * (am > ap ? am : ap);
    const T wf = T(tb1.w[q1]) * T(tb2.w[q2]) * ht1 * ht2;
    const T tau = s ? tau1 : tau0;
    T jmp[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) jmp[c] = tr[0][c] - tr[1][c];
    T* fo = FL + s * 8 * FP + pt;
    const T hth = T(0.5) * theta * nu * sg;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      // (grad u + grad u^T) e_D, component c, both sides
      T sym;
      if (c == D)
        sym = T(2) * (tr[0][3 + D] + tr[1][3 + D]);
      else if (c == T1)
        sym = tr[0][3 + c] + tr[0][6] + tr[1][3 + c] + tr[1][6];
      else
        sym = tr[0][3 + c] + tr[0][7] + tr[1][3 + c] + tr[1][7];
      const T fv = T(0.5) * (tr[0][c] * unm + tr[1][c] * unp) + T(0.5) * lam * jmp[c] - T(0.5) * nu * sym * sg +
                   tau * nu * jmp[c];
      // F_g[c][D] = -theta nu/2 (jmp_c + delta_cD jmp_D) sg
      const T Fn = (c == D) ? -T(2) * hth * jmp[D] : -hth * jmp[c];
      fo[c * FP] = wf * fv;
      fo[(3 + c) * FP] = wf * Fn;
      if constexpr (ENR && LE == 1) rt[c] += wf * (psim * fv + Fn * gpsim[D]);
      if constexpr (ENR && LE == 8) {
        // test functions psi N_B e_c: value psi N_B, d_D (psi N_B) = N_B d_D psi + psi d_D N_B
#pragma unroll
        for (int B = 0; B < 8; ++B)
          rt[c * 8 + B] += wf * (psim * nB[B] * fv + Fn * (nB[B] * gpsim[D] + psim * dB[D][B]));
      }
    }
    // F_g[D][T1] = -theta nu/2 jmp_T1 sg,  F_g[D][T2] = -theta nu/2 jmp_T2 sg
    const T Ft1 = -hth * jmp[T1], Ft2 = -hth * jmp[T2];
    fo[6 * FP] = wf * Ft1;
    fo[7 * FP] = wf * Ft2;
    if constexpr (ENR && LE == 1) rt[D] += wf * (Ft1 * gpsim[T1] + Ft2 * gpsim[T2]);
    if constexpr (ENR && LE == 8) {
#pragma unroll
      for (int B = 0; B < 8; ++B)
        rt[D * 8 + B] += wf * (Ft1 * (nB[B] * gpsim[T1] + psim * dB[T1][B]) +
                               Ft2 * (nB[B] * gpsim[T2] + psim * dB[T2][B]));
    }
  }
  __syncthreads();

  // Phase D1: lines along t2 transposed (q2 -> i2).  Tests 0-2: value test
  // S2^T fv_c (+ Sd2^T F[D][T2] / ht2 for c = D); 3: t1-derivative test
  // S2^T F[D][T1]; 4-6: normal-derivative test S2^T F[c][D].
  // (thread t: q1 = t & 7, face (t >> 3) & 1, test slot k = t >> 4; the
  // tests o = D, which add the Sd2 part, take slot 6, in wavefront 1 only)
  for (int t = tid; t < 7 * 16; t += nt) {
    const int q1 = t & 7, s = (t >> 3) & 1, k = t >> 4;
    if (q1 >= Q1) continue;
    const int o = k == 6 ? D : (k < D ? k : k + 1);
    const int fin = o < 3 ? o : (o == 3 ? 6 : o - 1);
    const T* a = FL + (s * 8 + fin) * FP + q1;
    T x[Q2];
#pragma unroll
    for (int q2 = 0; q2 < Q2; ++q2) x[q2] = a[q2 * Q1];
    T out[NP];
#pragma unroll
    for (int i2 = 0; i2 < NP; ++i2) {
      T acc = 0;
#pragma unroll
      for (int q2 = 0; q2 < Q2; ++q2) acc += T(tb2.S[q2][i2]) * x[q2];
      out[i2] = acc;
    }
    if (o == D) {
      const T* b = FL + (s * 8 + 7) * FP + q1;
#pragma unroll
      for (int q2 = 0; q2 < Q2; ++q2) x[q2] = b[q2 * Q1];
#pragma unroll
      for (int i2 = 0; i2 < NP; ++i2) {
        T acc = 0;
#pragma unroll
        for (int q2 = 0; q2 < Q2; ++q2) acc += T(tb2.Sd[q2][i2]) * x[q2];
        out[i2] += acc * iht2;
      }
    }
    T* dst = B1 + ((s * 7 + o) * Q1 + q1) * NP;
#pragma unroll
    for (int i2 = 0; i2 < NP; ++i2) dst[i2] = out[i2];
  }
  __syncthreads();

  // Phase D2: lines along t1 transposed (q1 -> i1): value test of u_c on the
  // face layer, and the normal-derivative test (to be spread along D).
  // (the value test of u_D, which adds the Sd1 part, comes last)
  for (int t = tid; t < 2 * 3 * 2 * NP; t += nt) {
    constexpr int N0 = 2 * 5 * NP;
    const bool last = t >= N0;
    const int tt = last ? t - N0 : t;
    const int i2 = tt % NP;
    int r = tt / NP;
    int kind, c, s;
    if (last) {
      kind = 0;
      c = D;
      s = r;
    } else {
      const int ci = r % 5;
      const int pi = ci < 2 * D ? ci : ci + 1;  // (c, kind) pairs as c * 2 + kind, skipping (D, 0)
      c = pi / 2;
      kind = pi % 2;
      s = r / 5;
    }
    const T* a = B1 + ((s * 7 + (kind ? 4 + c : c)) * Q1) * NP + i2;
    T x[Q1];
#pragma unroll
    for (int q1 = 0; q1 < Q1; ++q1) x[q1] = a[q1 * NP];
    T out[NP];
#pragma unroll
    for (int i1 = 0; i1 < NP; ++i1) {
      T acc = 0;
#pragma unroll
      for (int q1 = 0; q1 < Q1; ++q1) acc += T(tb1.S[q1][i1]) * x[q1];
      out[i1] = acc;
    }
    if (kind == 0 && c == D) {
      const T* b = B1 + ((s * 7 + 3) * Q1) * NP + i2;
#pragma unroll
      for (int q1 = 0; q1 < Q1; ++q1) x[q1] = b[q1 * NP];
#pragma unroll
      for (int i1 = 0; i1 < NP; ++i1) {
        T acc = 0;
#pragma unroll
        for (int q1 = 0; q1 < Q1; ++q1) acc += T(tb1.Sd[q1][i1]) * x[q1];
        out[i1] += acc * iht1;
      }
    }
    const T sc = kind ? ihd : T(1);
    T* dst = RB + ((s * 3 + c) * 2 + kind) * NP2 + NP * i2;
#pragma unroll
    for (int i1 = 0; i1 < NP; ++i1) dst[i1] = out[i1] * sc;
  }
  __syncthreads();

  // Phase E: spread onto the lines of nodes along D (value test on the face
  // layer, normal-derivative test on every layer); one thread per line.
  for (int t = tid; t < 3 * NP2; t += nt) {
    const int c = t / NP2, k = t - c * NP2;
    const T rv0 = RB[((0 * 3 + c) * 2 + 0) * NP2 + k], bn0 = RB[((0 * 3 + c) * 2 + 1) * NP2 + k];
    const T rv1 = RB[((1 * 3 + c) * 2 + 0) * NP2 + k], bn1 = RB[((1 * 3 + c) * 2 + 1) * NP2 + k];
    int base, stride;
    line_of<NP>(D, k % NP, k / NP, base, stride);
    T* dst = s_r + c * NP3 + base;
#pragma unroll
    for (int l = 0; l < NP; ++l) {
      T add = T(tbn.nd0[l]) * bn0 + T(tbn.nd1[l]) * bn1;
      if (l == 0) add += rv0;
      if (l == NP - 1) add += rv1;
      dst[l * stride] += add;
    }
  }
  __syncthreads();
}

// Curved cells: both faces of direction D with general normals.  Traces carry
// the full reference gradient (12 fields per side), mapped with the stored
// J^{-1} of each side at the face point; the gradient tests are pulled back
// to reference derivatives with the own side's J^{-1}.
template <typename T, int NP, int NQ, int NQY, bool ENR, int D>
__device__ __forceinline__ void vel_faces_dir_curved(const MeshDev& M, int64_t e, const T* s_u, const T* s_nl,
                                                     const T* s_nut, T* s_r, T* s_face, const T* s_ut,
                                                     const T* s_tab, int ex, int ey, int ez, int64_t enr, T rt[3]) {
  using Sh = VelShape<T, NP, NQ, NQY>;
  constexpr int T1 = D == 0 ? 1 : 0;
  constexpr int T2 = D == 2 ? 1 : 2;
  constexpr int Q1 = T1 == 1 ? NQY : NQ;
  constexpr int Q2 = T2 == 1 ? NQY : NQ;
  constexpr int FP = Q1 * Q2;
  constexpr int NP2 = Sh::NP2, NP3 = Sh::NP3;
  constexpr int QN = Q1 * NP;
  const int tid = threadIdx.x;
  constexpr int nt = 256;  // workgroup size of every velocity launch
  using TL = FaceTab<NP, NQ, NQY>;
  const T* S1 = s_tab + (T1 == 1 ? TL::Sy : TL::Sq);
  const T* Sd1 = s_tab + (T1 == 1 ? TL::Sdy : TL::Sdq);
  const T* S2 = s_tab + (T2 == 1 ? TL::Sy : TL::Sq);
  const T* Sd2 = s_tab + (T2 == 1 ? TL::Sdy : TL::Sdq);
  const T* nd0 = s_tab + TL::nd0;
  const T* nd1 = s_tab + TL::nd1;

  T* lay = s_face;                 // [s][c][val|d_n][NP2]
  T* A1 = lay + Sh::LAYO;          // [s][side][c][Sv|Sdv|Sn][q1][i2]
  T* fl = A1 + Sh::A1C;            // [s][12][pt]
  T* B1 = fl + Sh::FLC;            // [s][c][value|t1|normal][q1][i2]

  const FaceNb nb0 = face_nb(M, ex, ey, ez, D, 0), nb1 = face_nb(M, ex, ey, ez, D, 1);
  const bool wall0 = nb0.wall, wall1 = nb1.wall;

  for (int t = tid; t < 2 * 3 * NP2; t += nt) {
    const int s = t / (3 * NP2), rem = t - s * 3 * NP2;
    const int c = rem / NP2, k = rem - c * NP2;
    int base, stride;
    line_of<NP>(D, k % NP, k / NP, base, stride);
    const T* nd = s ? nd1 : nd0;
    const T* src = s_u + c * NP3 + base;
    T der = 0;
#pragma unroll
    for (int l = 0; l < NP; ++l) der += nd[l] * src[l * stride];
    lay[((s * 3 + c) * 2 + 0) * NP2 + k] = src[(s ? NP - 1 : 0) * stride];
    lay[((s * 3 + c) * 2 + 1) * NP2 + k] = der;
  }
  __syncthreads();

  for (int t = tid; t < 2 * 2 * 3 * 3 * QN; t += nt) {
    const int q1 = t % Q1;
    int r = t / Q1;
    const int i2 = r % NP;
    r /= NP;
    const int f = r % 3;
    r /= 3;
    const int c = r % 3;
    r /= 3;
    const int side = r % 2, s = r / 2;
    if (side == 1 && (s ? wall1 : wall0)) continue;
    const T* lv = (side == 0 ? lay + ((s * 3 + c) * 2) * NP2 : s_nl + (((2 * D + s) * 3 + c) * 2) * NP2) +
                  (f == 2 ? NP2 : 0) + NP * i2;
    const T* mat = (f == 1 ? Sd1 : S1) + q1 * NP;
    T acc = 0;
#pragma unroll
    for (int i1 = 0; i1 < NP; ++i1) acc += mat[i1] * lv[i1];
    A1[((((s * 2 + side) * 3 + c) * 3 + f) * Q1 + q1) * NP + i2] = acc;
  }
  __syncthreads();

  const T nu = T(M.nu), theta = T(M.theta);
  const int nqy_own = ENR ? NQY : NQ;
  for (int t = tid; t < 2 * FP; t += nt) {
    const int s = t / FP, pt = t - s * FP;
    const int q1 = pt % Q1, q2 = pt / Q1;
    const T sg = s ? T(1) : T(-1);
    const bool wall = s ? wall1 : wall0;
    const FaceNb& nb = s ? nb1 : nb0;
    const int f = 2 * D + s, fn = 2 * D + (1 - s);
    const double* go = M.geo + (e * M.geo_stride + psi_face_offset(NQ, nqy_own, f) + pt) * 10;
    T Jo[3][3], Jn[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int d = 0; d < 3; ++d) Jo[a][d] = T(go[3 * a + d]);
    const T wf = T(go[9]);
    T um[3], up[3], gm[3][3], gp[3][3];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      if (side == 1 && wall) continue;
      if (side == 1) {
        const int nqy_nb = nb.enr_nb >= 0 ? M.nq_wn : NQ;  // the neighbour's own point layout
        const double* gn = M.geo + (nb.enb * M.geo_stride + psi_face_offset(NQ, nqy_nb, fn) + pt) * 10;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int d = 0; d < 3; ++d) Jn[a][d] = T(gn[3 * a + d]);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T* a = A1 + (((s * 2 + side) * 3 + c) * 3) * QN + q1 * NP;
        T v = 0, d1 = 0, d2 = 0, dn = 0;
#pragma unroll
        for (int i2 = 0; i2 < NP; ++i2) {
          const T b2 = S2[q2 * NP + i2], bd2 = Sd2[q2 * NP + i2];
          v += b2 * a[i2];
          d1 += b2 * a[QN + i2];
          d2 += bd2 * a[i2];
          dn += b2 * a[2 * QN + i2];
        }
        T gr[3];
        gr[T1] = d1;
        gr[T2] = d2;
        gr[D] = dn;
        T* uo = side == 0 ? um : up;
        T(*go3)[3] = side == 0 ? gm : gp;
        uo[c] = v;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const T(*Jx)[3] = side == 0 ? Jo : Jn;
          go3[c][d] = gr[0] * Jx[0][d] + gr[1] * Jx[1][d] + gr[2] * Jx[2][d];
        }
      }
    }
    T psim = 0, gpsim[3] = {0, 0, 0};
    if (ENR) {
      const double* ps = M.psi + ((size_t)enr * M.psi_pts + M.psi_off[1 + f] + pt) * 4;
      psim = T(ps[0]);
      gpsim[0] = T(ps[1]);
      gpsim[1] = T(ps[2]);
      gpsim[2] = T(ps[3]);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        um[c] += psim * s_ut[c];
#pragma unroll
        for (int k = 0; k < 3; ++k) gm[c][k] += s_ut[c] * gpsim[k];
      }
    }
    if (wall) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        up[c] = -um[c];
#pragma unroll
        for (int k = 0; k < 3; ++k) gp[c][k] = gm[c][k];
      }
    } else if (nb.enr_nb >= 0) {
      const double* ps = M.psi + ((size_t)nb.enr_nb * M.psi_pts + M.psi_off[1 + fn] + pt) * 4;
      const T psip = T(ps[0]);
      const T gpp[3] = {T(ps[1]), T(ps[2]), T(ps[3])};
      const T* ut = s_nut + f * 3;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        up[c] += psip * ut[c];
#pragma unroll
        for (int k = 0; k < 3; ++k) gp[c][k] += ut[c] * gpp[k];
      }
    }
    T nv[3];
    {
      const T nr = sqrt(Jo[D][0] * Jo[D][0] + Jo[D][1] * Jo[D][1] + Jo[D][2] * Jo[D][2]);
#pragma unroll
      for (int d = 0; d < 3; ++d) nv[d] = sg * Jo[D][d] / nr;
    }
    const T tau = T(M.tauF[e * 6 + f]);
    const T unm = um[0] * nv[0] + um[1] * nv[1] + um[2] * nv[2];
    const T unp = up[0] * nv[0] + up[1] * nv[1] + up[2] * nv[2];
    const T am = unm < 0 ? -unm : unm, ap = unp < 0 ? -unp : unp;
    const T lam = T(2) * (am > ap ? am : ap);
    T jmp[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) jmp[c] = um[c] - up[c];
    T* fo = fl + s * 12 * FP + pt;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T visc = 0;
#pragma unroll
      for (int k = 0; k < 3; ++k) visc += (gm[c][k] + gm[k][c] + gp[c][k] + gp[k][c]) * nv[k];
      const T fv = T(0.5) * (um[c] * unm + up[c] * unp) + T(0.5) * lam * jmp[c] - T(0.5) * nu * visc +
                   tau * nu * jmp[c];
      T F[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) F[k] = -theta * nu * T(0.5) * (jmp[c] * nv[k] + jmp[k] * nv[c]);
      T Fr[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) Fr[a] = F[0] * Jo[a][0] + F[1] * Jo[a][1] + F[2] * Jo[a][2];
      fo[c * FP] = wf * fv;
      fo[(3 + c) * FP] = wf * Fr[T1];
      fo[(6 + c) * FP] = wf * Fr[T2];
      fo[(9 + c) * FP] = wf * Fr[D];
      if (ENR) rt[c] += wf * (psim * fv + F[0] * gpsim[0] + F[1] * gpsim[1] + F[2] * gpsim[2]);
    }
  }
  __syncthreads();

  for (int t = tid; t < 2 * 3 * QN; t += nt) {
    const int i2 = t % NP;
    int r = t / NP;
    const int q1 = r % Q1;
    r /= Q1;
    const int c = r % 3, s = r / 3;
    const T* fo = fl + s * 12 * FP + q1;
    T a0 = 0, a1 = 0, a3 = 0;
#pragma unroll
    for (int q2 = 0; q2 < Q2; ++q2) {
      const T b2 = S2[q2 * NP + i2], bd2 = Sd2[q2 * NP + i2];
      a0 += b2 * fo[c * FP + Q1 * q2] + bd2 * fo[(6 + c) * FP + Q1 * q2];
      a1 += b2 * fo[(3 + c) * FP + Q1 * q2];
      a3 += b2 * fo[(9 + c) * FP + Q1 * q2];
    }
    T* o = B1 + ((s * 3 + c) * 3) * QN + q1 * NP + i2;
    o[0] = a0;
    o[QN] = a1;
    o[2 * QN] = a3;
  }
  __syncthreads();

  for (int t = tid; t < 3 * NP2; t += nt) {
    const int c = t / NP2, k = t - c * NP2;
    const int i1 = k % NP, i2 = k / NP;
    T rv[2], bn[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const T* b = B1 + ((s * 3 + c) * 3) * QN + i2;
      T v = 0, n = 0;
#pragma unroll
      for (int q1 = 0; q1 < Q1; ++q1) {
        v += S1[q1 * NP + i1] * b[q1 * NP] + Sd1[q1 * NP + i1] * b[QN + q1 * NP];
        n += S1[q1 * NP + i1] * b[2 * QN + q1 * NP];
      }
      rv[s] = v;
      bn[s] = n;
    }
    int base, stride;
    line_of<NP>(D, i1, i2, base, stride);
    T* dst = s_r + c * NP3 + base;
#pragma unroll
    for (int l = 0; l < NP; ++l) {
      T add = nd0[l] * bn[0] + nd1[l] * bn[1];
      if (l == 0) add += rv[0];
      if (l == NP - 1) add += rv[1];
      dst[l * stride] += add;
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Affine (box) cells: face terms folded into the volume quadrature.
//
// Along every direction the velocity, its collocation gradient and every
// test function N_B, grad N_B restricted to a line of Gauss points are
// polynomials of degree <= k < n_q, so their values at the two faces are the
// exact extrapolations  f(0) = sum_q E0[q] f(g_q),  f(1) = sum_q E1[q] f(g_q).
// Hence
//   - the cell's own traces at the face Gauss points come from the volume
//     values and gradients at the Gauss points (one contraction along the
//     face normal), and
//   - the face test integrals  sum_f w_f (N_B fv + grad N_B : F_g)  equal
//     sum_q N_B(q) V(q) + grad N_B(q) : G_f(q)  with V and G_f the face fluxes
//     spread along the normal lines with E0 / E1, so they are added to the
//     volume flux G (and a value-test field V) before the transposed sweeps.
// Only the neighbour's traces still need a 2-D interpolation of its node
// layers.  With n = +-e_D the flux needs per side only u_c and the normal
// column of the symmetric gradient, s_c = (grad u + grad u^T)_{cD}, and
// F_g = -theta nu sym([u] (x) n) has the three distinct entries F_g[c][D] =
// F_g[D][c]: six fields per face point in both directions.
// ---------------------------------------------------------------------------

__host__ __device__ constexpr int aff_q1(int D, int NQ, int NQY) { return D == 0 ? NQY : NQ; }
__host__ __device__ constexpr int aff_q2(int D, int NQ, int NQY) { return D == 2 ? NQY : NQ; }
__host__ __device__ constexpr int aff_qd(int D, int NQ, int NQY) { return D == 1 ? NQY : NQ; }
constexpr int kAffFields = 6;
// start of face f = 2 D + s in the face-field array [face][field 0..5][point]
__host__ __device__ constexpr int aff_foff(int f, int NQ, int NQY) {
  int o = 0;
  for (int g = 0; g < f; ++g) o += kAffFields * aff_q1(g / 2, NQ, NQY) * aff_q2(g / 2, NQ, NQY);
  return o;
}

template <typename T, int NP, int NQ, int NQY>
struct AffShape {
  static constexpr int NP2 = NP * NP, NP3 = NP * NP * NP;
  static constexpr int NPTS = NQ * NQY * NQ;
  static constexpr int NL = 6 * 3 * 2 * NP2;             // neighbour layers [face][c][val|d_n][NP2]
  static constexpr int TA = 3 * NQ * NP * NP;             // interpolation temporaries (in the gradient region)
  static constexpr int TB = 3 * NQ * NQY * NP;
  // the neighbour layers go behind the temporaries when they fit, so that they
  // are stored in the phase of the last interpolation sweep
  static constexpr bool NL_EARLY = TA + TB + NL <= 9 * NPTS;
  static constexpr int VOL = 12 * NPTS;                   // u [c][pt], then grad u [c][d][pt]
  static constexpr int FLR = aff_foff(6, NQ, NQY);        // face fields
  static constexpr int FL = FLR > TB ? FLR : TB;          // (also the integration temporary)
  static constexpr int BYTES = (int)sizeof(T) * (3 * NP3 + VOL + FL);
  static constexpr bool fits = NL <= 9 * NPTS && BYTES <= 80 * 1024;
};

__device__ __forceinline__ int rotate_tid(int tofs) {
  const int t = (int)threadIdx.x;
  return t >= tofs ? t - tofs : t + 256 - tofs;
}

// Neighbour traces on the two faces of direction D at the face Gauss points,
// from the neighbour's node layers (value, physical normal derivative):
// fields 0-2 u_c, 3-5 s_c = d_D u_c + d_c u_D.  One thread per (face, field,
// q1): rows along t1 (per-lane rows of S1, S1' from LDS), then the t2 sweep
// with literal coefficients.  Items come in three kinds, in this order:
// u_c and s_D = 2 d_D u_D (one row sweep); s_T1 (adds the S1' row of u_D);
// s_T2 (adds the S2' sweep of the S1 rows of u_D).
template <typename T, int NP, int NQ, int NQY, int D>
__device__ __forceinline__ void aff_nb_traces(const T* s_nl, const T* s_tab, T* FL, bool wall0, bool wall1, T iht1,
                                              T iht2, int tofs) {
  constexpr int T1 = D == 0 ? 1 : 0;
  constexpr int T2 = D == 2 ? 1 : 2;
  constexpr int Q1 = aff_q1(D, NQ, NQY), Q2 = aff_q2(D, NQ, NQY), FP = Q1 * Q2;
  constexpr int NP2 = NP * NP;
  using TL = FaceTab<NP, NQ, NQY>;
  constexpr auto& tb2 = ct::tab<NP, Q2>;
  constexpr int N0 = 2 * 4 * Q1, N1 = N0 + 2 * Q1, N = N1 + 2 * Q1;
  constexpr int SROW = T1 == 1 ? TL::Sy : TL::Sq, SDROW = T1 == 1 ? TL::Sdy : TL::Sdq;
  for (int t = rotate_tid(tofs); t < N; t += 256) {
    const int kind = t < N0 ? 0 : (t < N1 ? 1 : 2);
    const int tt = kind == 0 ? t : (kind == 1 ? t - N0 : t - N1);
    const int q1 = tt % Q1;
    const int r = tt / Q1;
    const int j = kind == 0 ? (r & 3) : 0;
    const int s = kind == 0 ? (r >> 2) : r;
    if (s ? wall1 : wall0) continue;
    const T* lay = s_nl + (2 * D + s) * 3 * 2 * NP2;  // [c][val|d_n][NP2] of this face
    T m1[NP];
#pragma unroll
    for (int i1 = 0; i1 < NP; ++i1) m1[i1] = s_tab[SROW + q1 * NP + i1];
    // first row sweep: u_c (j < 3), s_D (j == 3), or the normal-derivative part of s_T1 / s_T2
    const int c = kind == 0 ? (j < 3 ? j : D) : (kind == 1 ? T1 : T2);
    const T* la = lay + (c * 2 + (kind == 0 && j < 3 ? 0 : 1)) * NP2;
    const T sc = (kind == 0 && j == 3) ? T(2) : T(1);
    T a[NP];
#pragma unroll
    for (int i2 = 0; i2 < NP; ++i2) {
      T acc = 0;
#pragma unroll
      for (int i1 = 0; i1 < NP; ++i1) acc += m1[i1] * la[i1 + NP * i2];
      a[i2] = acc * sc;
    }
    const int fo = kind == 0 ? (j < 3 ? j : 3 + D) : (kind == 1 ? 3 + T1 : 3 + T2);
    T* o = FL + aff_foff(2 * D + s, NQ, NQY) + fo * FP + q1;
    const T* lD = lay + (D * 2 + 0) * NP2;  // value layer of u_D
    if (kind == 1) {
      // + d_T1 u_D: S1' rows of the value layer of u_D
#pragma unroll
      for (int i1 = 0; i1 < NP; ++i1) m1[i1] = s_tab[SDROW + q1 * NP + i1];
#pragma unroll
      for (int i2 = 0; i2 < NP; ++i2) {
        T acc = 0;
#pragma unroll
        for (int i1 = 0; i1 < NP; ++i1) acc += m1[i1] * lD[i1 + NP * i2];
        a[i2] += acc * iht1;
      }
    }
    if (kind == 2) {
      // + d_T2 u_D: S2' sweep of the S1 rows of the value layer of u_D
      T b[NP];
#pragma unroll
      for (int i2 = 0; i2 < NP; ++i2) {
        T acc = 0;
#pragma unroll
        for (int i1 = 0; i1 < NP; ++i1) acc += m1[i1] * lD[i1 + NP * i2];
        b[i2] = acc * iht2;
      }
#pragma unroll
      for (int q2 = 0; q2 < Q2; ++q2) {
        T acc = 0;
#pragma unroll
        for (int i2 = 0; i2 < NP; ++i2) acc += T(tb2.S[q2][i2]) * a[i2] + T(tb2.Sd[q2][i2]) * b[i2];
        o[q2 * Q1] = acc;
      }
    } else {
#pragma unroll
      for (int q2 = 0; q2 < Q2; ++q2) {
        T acc = 0;
#pragma unroll
        for (int i2 = 0; i2 < NP; ++i2) acc += T(tb2.S[q2][i2]) * a[i2];
        o[q2 * Q1] = acc;
      }
    }
  }
}

// Numerical flux on face f = 2 D + S at every face Gauss point: own traces
// extrapolated from the volume values and gradients along the normal line,
// neighbour traces from FL (or the mirror state on a wall), then
// fv = {{u (x) u}} n + Lambda/2 [u] - {{2 nu eps(u)}} n + tau nu [u] and
// F_g[c][D] = -theta nu sym([u] (x) n)_{cD}, weighted by the face weight and
// written back into FL in place: [0..2] w fv_c, [3..5] w F_g[c][D].
// Enriched cells add the psi parts of both sides and the face terms of their
// enrichment test rows to rt.
template <typename T, int NP, int NQ, int NQY, bool ENR, int D, int S>
__device__ __forceinline__ void aff_flux(const MeshDev& M, const T* s_val, const T* s_grad, T* FL, const T* s_ut,
                                         const T* s_nut, bool wall, int64_t enr_nb, T tau, int64_t enr, T ht1, T ht2,
                                         T rt[3], int tofs) {
  constexpr int T1 = D == 0 ? 1 : 0;
  constexpr int T2 = D == 2 ? 1 : 2;
  constexpr int Q1 = aff_q1(D, NQ, NQY), Q2 = aff_q2(D, NQ, NQY), QD = aff_qd(D, NQ, NQY), FP = Q1 * Q2;
  constexpr int NPTS = NQ * NQY * NQ;
  constexpr int SD = D == 0 ? 1 : (D == 1 ? NQ : NQ * NQY);  // Gauss-point stride along D
  constexpr int f = 2 * D + S;
  constexpr auto& tbd = ct::tab<NP, QD>;
  constexpr auto& tb1 = ct::tab<NP, Q1>;
  constexpr auto& tb2 = ct::tab<NP, Q2>;
  const T nu = T(M.nu), theta = T(M.theta);
  const T sg = S ? T(1) : T(-1);
  for (int pt = rotate_tid(tofs); pt < FP; pt += 256) {
    const int q1 = pt % Q1, q2 = pt / Q1;
    const int base = D == 0 ? NQ * (q1 + NQY * q2) : (D == 1 ? q1 + NQ * NQY * q2 : q1 + NQ * q2);
    // own traces: u_c and s_c = d_D u_c + d_c u_D (grad u at [c][d])
    T um[3], sm[3], up[3], sp[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T* pu = s_val + c * NPTS + base;
      const T* pa = s_grad + (c * 3 + D) * NPTS + base;
      const T* pb = s_grad + (D * 3 + c) * NPTS + base;
      T au = 0, as = 0;
#pragma unroll
      for (int q = 0; q < QD; ++q) {
        const T e = T(S ? tbd.E1[q] : tbd.E0[q]);
        au += e * pu[q * SD];
        as += e * (c == D ? T(2) * pa[q * SD] : pa[q * SD] + pb[q * SD]);
      }
      um[c] = au;
      sm[c] = as;
    }
    T* fo = FL + aff_foff(f, NQ, NQY) + pt;
    if (!wall) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        up[c] = fo[c * FP];
        sp[c] = fo[(3 + c) * FP];
      }
    }
    T psim = 0, gpsim[3] = {0, 0, 0};
    if (ENR) {
      const double* ps = M.psi + ((size_t)enr * M.psi_pts + M.psi_off[1 + f] + pt) * 4;
      psim = T(ps[0]);
      gpsim[0] = T(ps[1]);
      gpsim[1] = T(ps[2]);
      gpsim[2] = T(ps[3]);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        um[c] += psim * s_ut[c];
        sm[c] += s_ut[c] * gpsim[D] + s_ut[D] * gpsim[c];
      }
    }
    if (wall) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        up[c] = -um[c];
        sp[c] = sm[c];
      }
    } else if (enr_nb >= 0) {
      const double* ps = M.psi + ((size_t)enr_nb * M.psi_pts + M.psi_off[1 + 2 * D + (1 - S)] + pt) * 4;
      const T psip = T(ps[0]);
      const T gpp[3] = {T(ps[1]), T(ps[2]), T(ps[3])};
      const T* ut = s_nut + f * 3;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        up[c] += psip * ut[c];
        sp[c] += ut[c] * gpp[D] + ut[D] * gpp[c];
      }
    }
    // n = sg e_D
    const T unm = sg * um[D], unp = sg * up[D];
    const T am = unm < 0 ? -unm : unm, ap = unp < 0 ? -unp : unp;
    const T lam = T(2) * (am > ap ? am : ap);
    const T wf = T(tb1.w[q1]) * T(tb2.w[q2]) * ht1 * ht2;
    const T hth = T(0.5) * theta * nu * sg;
    T Fg[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T jmp = um[c] - up[c];
      const T fv = T(0.5) * (um[c] * unm + up[c] * unp) + T(0.5) * lam * jmp - T(0.5) * nu * sg * (sm[c] + sp[c]) +
                   tau * nu * jmp;
      // F_g[c][D] = -theta nu/2 (jmp_c n_D + jmp_D n_c)
      Fg[c] = (c == D ? -T(2) : -T(1)) * hth * jmp;
      fo[c * FP] = wf * fv;
      fo[(3 + c) * FP] = wf * Fg[c];
      if (ENR) rt[c] += wf * (psim * fv + Fg[c] * gpsim[D]);
    }
    if (ENR) rt[D] += wf * (Fg[T1] * gpsim[T1] + Fg[T2] * gpsim[T2]);
  }
}

// Spread the weighted fluxes of face f = 2 D + S onto the Gauss point
// (qx, qy, qz) of the normal line through it: V_c += e fv_c, G[c][D] += e
// F_g[c][D] and G[D][c] += e F_g[D][c] (c != D), with e the extrapolation
// weight of the point's position along D (s_ext).
template <typename T, int NQ, int NQY, int D, int S>
__device__ __forceinline__ void aff_spread(const T* FL, const T* s_ext, int qx, int qy, int qz, T V[3], T G[3][3]) {
  constexpr int Q1 = aff_q1(D, NQ, NQY), FP = Q1 * aff_q2(D, NQ, NQY);
  const int qd = D == 0 ? qx : (D == 1 ? qy : qz);
  const int q1 = D == 0 ? qy : qx;
  const int q2 = D == 2 ? qy : qz;
  // s_ext: [rule NQ | NQY][E0 | E1][8]
  const T e = s_ext[((D == 1 ? 1 : 0) * 2 + S) * 8 + qd];
  const T* F = FL + aff_foff(2 * D + S, NQ, NQY) + q1 + Q1 * q2;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    V[c] += e * F[c * FP];
    const T g = e * F[(3 + c) * FP];
    G[c][D] += g;
    if (c != D) G[D][c] += g;
  }
}

template <typename T, int NP, int NQ, int NQY, bool ENR>
__device__ __forceinline__ void vel_cell_affine(const MeshDev& M, const T* __restrict__ u, T* __restrict__ r, int b,
                                                int layer_lo, int nlayers) {
  using Sh = AffShape<T, NP, NQ, NQY>;
  constexpr int NP3 = Sh::NP3, NPTS = Sh::NPTS;
  __shared__ T s_r0[3 * NP3];
  __shared__ T s_vol[Sh::VOL];
  __shared__ T s_fl[Sh::FL];
  __shared__ T s_ut[3];
  __shared__ T s_nut[18];
  __shared__ T s_red[3 * 4];
  __shared__ T s_tab[FaceTab<NP, NQ, NQY>::size];
  __shared__ T s_ext[32];
  const int tid = threadIdx.x;
  constexpr int nt = 256;  // workgroup size of every velocity launch

  const int ex = b % M.nx;
  const int t0 = b / M.nx;
  int ey, ez;
  int64_t enr = -1;
  if (ENR) {
    const int slot = t0 % M.nslots;
    ez = t0 / M.nslots;
    ey = (slot == M.lower_slot) ? 0 : M.ny - 1;
    enr = b;
  } else {
    ey = layer_lo + t0 % nlayers;
    ez = t0 / nlayers;
  }
  const int64_t e = ex + (int64_t)M.nx * (ey + (int64_t)M.ny * ez);
  const T hx = T(M.hx), hz = T(M.hz), hy = T(M.hy[ey]);
  const T ix = T(M.ihx), iy = T(M.ihy[ey]), iz = T(M.ihz);

  const double* tab = M.tab;
  using Sx = ct::MatS<NP, NQ>;
  using Sy = ct::MatS<NP, NQY>;
  using Dx = ct::MatD<NP, NQ>;
  using Dy = ct::MatD<NP, NQY>;
  constexpr auto& tbx = ct::tab<NP, NQ>;
  constexpr auto& tby = ct::tab<NP, NQY>;
  constexpr bool MEM = sizeof(T) == 8;
  constexpr TabLayout TL = tab_layout(NP, NQ, NQY);
  const double* mSx = tab + TL.S;
  const double* mDx = tab + TL.D;
  const double* mSy = tab + (ENR ? TL.Sy : TL.S);
  const double* mDy = tab + (ENR ? TL.Dy : TL.D);

  T* s_u = s_r0;
  T* s_val = s_vol;             // [c][pt]
  T* s_grad = s_vol + 3 * NPTS; // [c][d][pt]
  T* tA = s_grad;               // (NQ, NP, NP) x 3
  T* tB = tA + Sh::TA;          // (NQ, NQY, NP) x 3
  T* s_nl = Sh::NL_EARLY ? tB + Sh::TB : s_grad;
  for (int i = tid; i < 3 * NP3; i += nt) s_u[i] = u[e * 3 * NP3 + i];
  if (ENR && tid < 3) s_ut[tid] = u[M.enr_off + enr * 3 + tid];
  NbLines<T, NP> nbl;
  nb_fetch<T, NP>(M, u, ex, ey, ez, nbl);
  load_face_tab<T, NP, NQ, NQY, ENR>(tab, s_tab);
  if (tid < 32) {
    const int rule = tid >> 4, side = (tid >> 3) & 1, q = tid & 7;
    double v = 0.0;
    if (rule == 0 && q < NQ) v = side ? tbx.E1[q < NQ ? q : 0] : tbx.E0[q < NQ ? q : 0];
    if (rule == 1 && q < NQY) v = side ? tby.E1[q < NQY ? q : 0] : tby.E0[q < NQY ? q : 0];
    s_ext[tid] = T(v);
  }
  // faces: neighbours and penalties (uniform over the workgroup)
  const FaceNb nb[6] = {face_nb(M, ex, ey, ez, 0, 0), face_nb(M, ex, ey, ez, 0, 1), face_nb(M, ex, ey, ez, 1, 0),
                        face_nb(M, ex, ey, ez, 1, 1), face_nb(M, ex, ey, ez, 2, 0), face_nb(M, ex, ey, ez, 2, 1)};
  const T ihown[3] = {ix, iy, iz};
  T tau[6];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int D = f >> 1;
    const T ihd = ihown[D];
    if (nb[f].wall) tau[f] = T(M.pen * M.wall_mult) * ihd;
    else if (D != 1) tau[f] = T(M.pen) * ihd;
    else {
      const T ihn = T(M.ihy[nb[f].nidx1]);
      tau[f] = T(M.pen) * (ihd > ihn ? ihd : ihn);
    }
  }
  const int y0 = ey == 0 ? M.ny - 1 : ey - 1, y1 = ey + 1 == M.ny ? 0 : ey + 1;
  __syncthreads();

  // values at the Gauss points: x, y, z interpolation sweeps; the
  // neighbours' node layers go to LDS with the last one (or right after it)
  sweep_c<0, NP, NP, NP, NQ, false, false, Sx, 256, MEM>(s_u, NP3, tA, NQ * NP * NP, T(1), 3, 0, mSx);
  __syncthreads();
  sweep_c<1, NQ, NP, NP, NQY, false, false, Sy, 256, MEM>(tA, NQ * NP * NP, tB, NQ * NQY * NP, T(1), 3, 0, mSy);
  __syncthreads();
  sweep_c<2, NQ, NQY, NP, NQ, false, false, Sx, 256, MEM>(tB, NQ * NQY * NP, s_val, NPTS, T(1), 3, 0, mSx);
  if (!Sh::NL_EARLY) __syncthreads();
  nb_store<T, NP, NQ, false>(M, nbl, s_nl, s_nut, ex, ey, ez, ix, iz, T(M.ihy[y0]), T(M.ihy[y1]));
  __syncthreads();

  // neighbour traces of all six faces (each direction on whole wavefronts)
  T* FL = s_fl;
  aff_nb_traces<T, NP, NQ, NQY, 0>(s_nl, s_tab, FL, nb[0].wall, nb[1].wall, iy, iz, 0);
  aff_nb_traces<T, NP, NQ, NQY, 1>(s_nl, s_tab, FL, nb[2].wall, nb[3].wall, ix, iz, 128);
  aff_nb_traces<T, NP, NQ, NQY, 2>(s_nl, s_tab, FL, nb[4].wall, nb[5].wall, ix, iy, 64);
  __syncthreads();

  // gradients by collocation through the Gauss points (over the layers)
  constexpr int NLG = 3 * NPTS / NQ;
  constexpr int NLY = 3 * NPTS / NQY;
  sweep_c<0, NQ, NQY, NQ, NQ, false, false, Dx, 256, MEM>(s_val, NPTS, s_grad + 0 * NPTS, 3 * NPTS, ix, 3, 0, mDx);
  sweep_c<1, NQ, NQY, NQ, NQY, false, false, Dy, 256, MEM>(s_val, NPTS, s_grad + 1 * NPTS, 3 * NPTS, iy, 3,
                                                           NLG % 256, mDy);
  sweep_c<2, NQ, NQY, NQ, NQ, false, false, Dx, 256, MEM>(s_val, NPTS, s_grad + 2 * NPTS, 3 * NPTS, iz, 3,
                                                          (NLG + NLY) % 256, mDx);
  __syncthreads();

  // numerical fluxes of all six faces (in place; one face per wavefront)
  T rt[3] = {0, 0, 0};
  aff_flux<T, NP, NQ, NQY, ENR, 0, 0>(M, s_val, s_grad, FL, s_ut, s_nut, nb[0].wall, nb[0].enr_nb, tau[0], enr, hy,
                                      hz, rt, 0);
  aff_flux<T, NP, NQ, NQY, ENR, 0, 1>(M, s_val, s_grad, FL, s_ut, s_nut, nb[1].wall, nb[1].enr_nb, tau[1], enr, hy,
                                      hz, rt, 64);
  aff_flux<T, NP, NQ, NQY, ENR, 1, 0>(M, s_val, s_grad, FL, s_ut, s_nut, nb[2].wall, nb[2].enr_nb, tau[2], enr, hx,
                                      hz, rt, 128);
  aff_flux<T, NP, NQ, NQY, ENR, 1, 1>(M, s_val, s_grad, FL, s_ut, s_nut, nb[3].wall, nb[3].enr_nb, tau[3], enr, hx,
                                      hz, rt, 192);
  aff_flux<T, NP, NQ, NQY, ENR, 2, 0>(M, s_val, s_grad, FL, s_ut, s_nut, nb[4].wall, nb[4].enr_nb, tau[4], enr, hx,
                                      hy, rt, 128);
  aff_flux<T, NP, NQ, NQY, ENR, 2, 1>(M, s_val, s_grad, FL, s_ut, s_nut, nb[5].wall, nb[5].enr_nb, tau[5], enr, hx,
                                      hy, rt, 192);
  __syncthreads();

  // pointwise flux G = w (2 nu eps(u) - u (x) u), plus the face fluxes spread
  // along the normal lines (gradient tests into G, value tests into V)
  const T nu = T(M.nu);
  const T vol = hx * hy * hz;
  for (int pt = tid; pt < NPTS; pt += nt) {
    const int qx = pt % NQ, qy = (pt / NQ) % NQY, qz = pt / (NQ * NQY);
    const T wq = T(tbx.w[qx]) * T(tby.w[qy]) * T(tbx.w[qz]) * vol;
    T uu[3], gg[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      uu[c] = s_val[c * NPTS + pt];
#pragma unroll
      for (int d = 0; d < 3; ++d) gg[c][d] = s_grad[(c * 3 + d) * NPTS + pt];
    }
    T gps[3] = {0, 0, 0};
    if (ENR) {
      const double* ps = M.psi + ((size_t)enr * M.psi_pts + pt) * 4;
      const T psv = T(ps[0]);
      gps[0] = T(ps[1]);
      gps[1] = T(ps[2]);
      gps[2] = T(ps[3]);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        uu[c] += psv * s_ut[c];
#pragma unroll
        for (int d = 0; d < 3; ++d) gg[c][d] += s_ut[c] * gps[d];
      }
    }
    T G[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        G[c][d] = wq * (nu * (gg[c][d] + gg[d][c]) - uu[c] * uu[d]);
        if (ENR) rt[c] += G[c][d] * gps[d];
      }
    T V[3] = {0, 0, 0};
    aff_spread<T, NQ, NQY, 0, 0>(FL, s_ext, qx, qy, qz, V, G);
    aff_spread<T, NQ, NQY, 0, 1>(FL, s_ext, qx, qy, qz, V, G);
    aff_spread<T, NQ, NQY, 1, 0>(FL, s_ext, qx, qy, qz, V, G);
    aff_spread<T, NQ, NQY, 1, 1>(FL, s_ext, qx, qy, qz, V, G);
    aff_spread<T, NQ, NQY, 2, 0>(FL, s_ext, qx, qy, qz, V, G);
    aff_spread<T, NQ, NQY, 2, 1>(FL, s_ext, qx, qy, qz, V, G);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      s_val[c * NPTS + pt] = V[c];
#pragma unroll
      for (int d = 0; d < 3; ++d) s_grad[(c * 3 + d) * NPTS + pt] = G[c][d];
    }
  }
  __syncthreads();

  // integrate: W = sum_d D_d^T G_d / h_d + V, then transposed interpolation
  sweep_c_inplace<0, NQ, NQY, NQ, true, Dx, 256, MEM>(s_grad + 0 * NPTS, 3 * NPTS, ix, 3, 0, mDx);
  sweep_c_inplace<1, NQ, NQY, NQ, true, Dy, 256, MEM>(s_grad + 1 * NPTS, 3 * NPTS, iy, 3, NLG % 256, mDy);
  __syncthreads();
  {
    T* tB2 = s_fl;                        // (NQ, NQY, NP) x 3
    T* tA2 = s_grad;                      // (NQ, NP, NP) x 3
    for (int t = tid; t < 3 * NQ * NQY; t += nt) {
      const int c = t / (NQ * NQY), pq = t - c * (NQ * NQY);  // pq = qx + NQ qy
      const T* gz = s_grad + (c * 3 + 2) * NPTS + pq;
      const T* wx = s_grad + (c * 3 + 0) * NPTS + pq;
      const T* wy = s_grad + (c * 3 + 1) * NPTS + pq;
      const T* vv = s_val + c * NPTS + pq;
      T g[NQ], w[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) g[q] = gz[q * NQ * NQY];
#pragma unroll
      for (int q = 0; q < NQ; ++q) w[q] = wx[q * NQ * NQY] + wy[q * NQ * NQY] + vv[q * NQ * NQY];
#pragma unroll
      for (int m = 0; m < NQ; ++m) {
        T sacc = 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) sacc += T(MEM ? mDx[q * NQ + m] : tbx.D[q][m]) * g[q];
        w[m] += iz * sacc;
      }
      T* o = tB2 + c * (NQ * NQY * NP) + pq;
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        T sacc = 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) sacc += T(MEM ? mSx[q * NP + i] : tbx.S[q][i]) * w[q];
        o[i * NQ * NQY] = sacc;
      }
    }
    __syncthreads();
    sweep_c<1, NQ, NQY, NP, NP, true, false, Sy, 256, MEM>(tB2, NQ * NQY * NP, tA2, NQ * NP * NP, T(1), 3, 0, mSy);
    __syncthreads();
    T* s_r = s_r0;
    sweep_c<0, NQ, NP, NP, NP, true, false, Sx, 256, MEM>(tA2, NQ * NP * NP, s_r, NP3, T(1), 3, 0, mSx);
    __syncthreads();
    for (int i = tid; i < 3 * NP3; i += nt) r[e * 3 * NP3 + i] = s_r[i];
  }
  if (ENR) {
    block_sum3(rt, s_red);
    if (tid < 3) r[M.enr_off + enr * 3 + tid] = rt[0];
  }
}

// One cell: block-local index b within its launch (regular cells: layer range
// [layer_lo, layer_lo + nlayers); enriched cells: the enriched index).
template <typename T, int NP, int NQ, int NQY, bool ENR, bool CURVED, bool MS = false, int LE = 1>
__device__ __forceinline__ void vel_cell_general(const MeshDev& M, const T* __restrict__ u, T* __restrict__ r, int b,
                                                 int layer_lo, int nlayers) {
  static_assert(LE == 1 || (LE == 8 && !CURVED), "degree-1 weights: flat cells");
  using Sh = VelShape<T, NP, NQ, NQY>;
  constexpr int NP3 = Sh::NP3, NPTS = Sh::NPTS;
  __shared__ T s_u[3 * NP3];
  __shared__ T s_r[3 * NP3];
  __shared__ T s_big[Sh::BIG];
  __shared__ T s_ut[3 * LE];      // enrichment coefficients [c][B]
  __shared__ T s_nut[18 * LE];    // the neighbours' ones [face][c][B]
  __shared__ T s_red[3 * LE * 4];
  __shared__ T s_tab[FaceTab<NP, NQ, NQY>::size];
  const int tid = threadIdx.x;
  constexpr int nt = 256;  // workgroup size of every velocity launch

  const int ex = b % M.nx;
  const int t0 = b / M.nx;
  int ey, ez;
  int64_t enr = -1;
  if (ENR) {
    const int slot = t0 % M.nslots;
    ez = t0 / M.nslots;
    ey = (slot == M.lower_slot) ? 0 : M.ny - 1;
    enr = b;
  } else {
    ey = layer_lo + t0 % nlayers;
    ez = t0 / nlayers;
  }
  const int64_t e = ex + (int64_t)M.nx * (ey + (int64_t)M.ny * ez);
  const T hx = T(M.hx), hz = T(M.hz), hy = T(M.hy[ey]);
  // sweeps produce physical derivatives on affine cells, reference ones on curved cells
  const T ix = CURVED ? T(1) : T(M.ihx), iy = CURVED ? T(1) : T(M.ihy[ey]), iz = CURVED ? T(1) : T(M.ihz);

  const double* tab = M.tab;
  // volume sweep matrices: compile-time tables (x and z use the NQ rule, y
  // the NQY rule, which is NQ outside the enriched layer)
  using Sx = ct::MatS<NP, NQ>;
  using Sy = ct::MatS<NP, NQY>;
  using Dx = ct::MatD<NP, NQ>;
  using Dy = ct::MatD<NP, NQY>;
  constexpr auto& tbx = ct::tab<NP, NQ>;
  constexpr auto& tby = ct::tab<NP, NQY>;
  // FP64 sweeps read the same tables from the mesh's table block (see sweep_c)
  constexpr bool MEM = sizeof(T) == 8;
  constexpr TabLayout TL = tab_layout(NP, NQ, NQY);
  const double* mSx = tab + TL.S;
  const double* mDx = tab + TL.D;
  const double* mSy = tab + (ENR ? TL.Sy : TL.S);
  const double* mDy = tab + (ENR ? TL.Dy : TL.D);

  for (int i = tid; i < 3 * NP3; i += nt) s_u[i] = u[e * 3 * NP3 + i];
  if (ENR && tid < 3 * LE) s_ut[tid] = u[M.enr_off + enr * 3 * LE + tid];
  NbLines<T, NP> nbl;
  nb_fetch<T, NP, LE>(M, u, ex, ey, ez, nbl);
  // psi and grad psi at the thread's volume points (enriched cells), loaded
  // with the cell so that their latency overlaps the sweeps
  constexpr int NPASS = (NPTS + nt - 1) / nt;
  T pfv[NPASS][4];
  if constexpr (ENR && !MS) {
#pragma unroll
    for (int kp = 0; kp < NPASS; ++kp) {
      const int pt = tid + kp * nt;
#pragma unroll
      for (int j = 0; j < 4; ++j) pfv[kp][j] = 0;
      if (pt < NPTS) {
        const double* ps = M.psi + ((size_t)enr * M.psi_pts + pt) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) pfv[kp][j] = T(ps[j]);
      }
    }
  }
  if (CURVED) load_face_tab<T, NP, NQ, NQY, ENR>(tab, s_tab);
  __syncthreads();

  T* s_val = s_big;             // [c][pt]
  T* s_grad = s_big + 3 * NPTS; // [c][d][pt]
  // values at the Gauss points: x, y, z interpolation sweeps
  {
    T* tA = s_grad;                       // (NQ, NP, NP) x 3
    T* tB = tA + 3 * NQ * NP * NP;        // (NQ, NQY, NP) x 3
    sweep_c<0, NP, NP, NP, NQ, false, false, Sx, 256, MEM>(s_u, NP3, tA, NQ * NP * NP, T(1), 3, 0, mSx);
    __syncthreads();
    sweep_c<1, NQ, NP, NP, NQY, false, false, Sy, 256, MEM>(tA, NQ * NP * NP, tB, NQ * NQY * NP, T(1), 3, 0, mSy);
    __syncthreads();
    sweep_c<2, NQ, NQY, NP, NQ, false, false, Sx, 256, MEM>(tB, NQ * NQY * NP, s_val, NPTS, T(1), 3, 0, mSx);
    __syncthreads();
  }
  // gradients by collocation through the Gauss points
  // (the three sweeps are independent: rotated thread assignments pack them)
  constexpr int NLG = 3 * NPTS / NQ;   // lines per x- or z-sweep (3 components)
  constexpr int NLY = 3 * NPTS / NQY;  // lines per y-sweep
  sweep_c<0, NQ, NQY, NQ, NQ, false, false, Dx, 256, MEM>(s_val, NPTS, s_grad + 0 * NPTS, 3 * NPTS, ix, 3, 0, mDx);
  sweep_c<1, NQ, NQY, NQ, NQY, false, false, Dy, 256, MEM>(s_val, NPTS, s_grad + 1 * NPTS, 3 * NPTS, iy, 3,
                                                           NLG % 256, mDy);
  sweep_c<2, NQ, NQY, NQ, NQ, false, false, Dx, 256, MEM>(s_val, NPTS, s_grad + 2 * NPTS, 3 * NPTS, iz, 3,
                                                          (NLG + NLY) % 256, mDx);
  __syncthreads();

  // pointwise flux G = 2 nu eps(u) - u (x) u, times the quadrature weight
  T rt[3 * LE];
#pragma unroll
  for (int i = 0; i < 3 * LE; ++i) rt[i] = 0;
  const T nu = T(M.nu);
  const T vol = hx * hy * hz;
#pragma unroll
  for (int kp = 0; kp < NPASS; ++kp) {
    const int pt = tid + kp * nt;
    if (pt >= NPTS) break;
    const int qx = pt % NQ, qy = (pt / NQ) % NQY, qz = pt / (NQ * NQY);
    T wq, Ji[3][3];
    if (CURVED) {
      const double* g = M.geo + (e * M.geo_stride + pt) * 10;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int d = 0; d < 3; ++d) Ji[a][d] = T(g[3 * a + d]);
      wq = T(g[9]);
    } else {
      wq = T(tbx.w[qx]) * T(tby.w[qy]) * T(tbx.w[qz]) * vol;
    }
    T uu[3], gg[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      uu[c] = s_val[c * NPTS + pt];
      if (CURVED) {
        T gr[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) gr[a] = s_grad[(c * 3 + a) * NPTS + pt];
#pragma unroll
        for (int d = 0; d < 3; ++d) gg[c][d] = gr[0] * Ji[0][d] + gr[1] * Ji[1][d] + gr[2] * Ji[2][d];
      } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) gg[c][d] = s_grad[(c * 3 + d) * NPTS + pt];
      }
    }
    if constexpr (MS) {
      // multiscale viscous volume terms (eq. viscous_multiscale): polynomial
      // tests against 2 nu eps(u_bar) + 2 nuhat eps(u~), nuhat the limited
      // viscosity of eq. minvt; enrichment tests against 2 (nu + nu_t) eps(u~)
      T gt[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
      T gps[3] = {0, 0, 0}, nt = nu, nhat = nu, psv = 0;
      T nB[LE], dB[3][LE];
      if (ENR) {
        const double* ps = M.psi + ((size_t)enr * M.psi_pts + pt) * 4;
        psv = T(ps[0]);
        gps[0] = T(ps[1]);
        gps[1] = T(ps[2]);
        gps[2] = T(ps[3]);
        nt = nu + T(M.nut[(size_t)enr * M.psi_pts + pt]);
        const T lim = T(2) * sqrt(nu * nt);
        nhat = nt < lim ? nt : lim;
        if constexpr (LE == 1) {
#pragma unroll
          for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int d = 0; d < 3; ++d) gt[c][d] = s_ut[c] * gps[d];
        } else {
          const T xi[3] = {T(tbx.g[qx]), T(tby.g[qy]), T(tbx.g[qz])}, ih3[3] = {ix, iy, iz};
          T L[3], dL[3][3];
          vertex_fns(xi, ih3, nB, dB);
          vertex_weight(s_ut, nB, dB, L, dL);
#pragma unroll
          for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int d = 0; d < 3; ++d) gt[c][d] = L[c] * gps[d] + psv * dL[c][d];
        }
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        T sv[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const T st = gt[c][d] + gt[d][c];
          sv[d] = st;
          if (ENR && LE == 1) rt[c] += wq * nt * st * gps[d];
          s_grad[(c * 3 + d) * NPTS + pt] = wq * (nu * (gg[c][d] + gg[d][c]) + nhat * st);
        }
        if constexpr (ENR && LE == 8) {
          // eps(phi e_c) : F = sum_d d_d phi F[c][d], phi = psi N_B
#pragma unroll
          for (int B = 0; B < 8; ++B) {
            T a = 0;
#pragma unroll
            for (int d = 0; d < 3; ++d) a += sv[d] * (nB[B] * gps[d] + psv * dB[d][B]);
            rt[c * 8 + B] += wq * nt * a;
          }
        }
      }
      continue;
    }
    T gps[3] = {0, 0, 0}, psv = 0;
    T nB[LE], dB[3][LE];  // degree-1 weights: vertex functions at the point
    if (ENR) {
      psv = pfv[kp][0];
      gps[0] = pfv[kp][1];
      gps[1] = pfv[kp][2];
      gps[2] = pfv[kp][3];
      if constexpr (LE == 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          uu[c] += psv * s_ut[c];
#pragma unroll
          for (int d = 0; d < 3; ++d) gg[c][d] += s_ut[c] * gps[d];
        }
      } else {
        const T xi[3] = {T(tbx.g[qx]), T(tby.g[qy]), T(tbx.g[qz])}, ih3[3] = {ix, iy, iz};
        T L[3], dL[3][3];
        vertex_fns(xi, ih3, nB, dB);
        vertex_weight(s_ut, nB, dB, L, dL);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          uu[c] += psv * L[c];
#pragma unroll
          for (int d = 0; d < 3; ++d) gg[c][d] += L[c] * gps[d] + psv * dL[c][d];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T G[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        G[d] = wq * (nu * (gg[c][d] + gg[d][c]) - uu[c] * uu[d]);
        if (ENR && LE == 1) rt[c] += G[d] * gps[d];
      }
      if constexpr (ENR && LE == 8) {
        // grad (psi N_B) = N_B grad psi + psi grad N_B
        const T a = G[0] * gps[0] + G[1] * gps[1] + G[2] * gps[2];
#pragma unroll
        for (int B = 0; B < 8; ++B)
          rt[c * 8 + B] += nB[B] * a + psv * (G[0] * dB[0][B] + G[1] * dB[1][B] + G[2] * dB[2][B]);
      }
#pragma unroll
      for (int a = 0; a < 3; ++a)
        s_grad[(c * 3 + a) * NPTS + pt] = CURVED ? G[0] * Ji[a][0] + G[1] * Ji[a][1] + G[2] * Ji[a][2] : G[a];
    }
  }
  __syncthreads();

  // integrate: W = sum_d D_d^T G_d / h_d, then transposed interpolation.
  // The x and y parts are formed in place (one phase); each z line then adds
  // its own D_z^T G_z to them and applies S_z^T directly.
  sweep_c_inplace<0, NQ, NQY, NQ, true, Dx, 256, MEM>(s_grad + 0 * NPTS, 3 * NPTS, ix, 3, 0, mDx);
  sweep_c_inplace<1, NQ, NQY, NQ, true, Dy, 256, MEM>(s_grad + 1 * NPTS, 3 * NPTS, iy, 3, NLG % 256, mDy);
  __syncthreads();
  {
    T* tB = s_val;                        // (NQ, NQY, NP) x 3 (u is no longer needed)
    T* tA = s_grad;                       // (NQ, NP, NP) x 3
    constexpr auto& tbz = ct::tab<NP, NQ>;
    for (int t = tid; t < 3 * NQ * NQY; t += nt) {
      const int c = t / (NQ * NQY), pq = t - c * (NQ * NQY);  // pq = qx + NQ qy
      const T* gz = s_grad + (c * 3 + 2) * NPTS + pq;
      const T* wx = s_grad + (c * 3 + 0) * NPTS + pq;
      const T* wy = s_grad + (c * 3 + 1) * NPTS + pq;
      T g[NQ], w[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) g[q] = gz[q * NQ * NQY];
#pragma unroll
      for (int q = 0; q < NQ; ++q) w[q] = wx[q * NQ * NQY] + wy[q * NQ * NQY];
#pragma unroll
      for (int m = 0; m < NQ; ++m) {
        T sacc = 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) sacc += T(MEM ? mDx[q * NQ + m] : tbz.D[q][m]) * g[q];
        w[m] += iz * sacc;
      }
      T* o = tB + c * (NQ * NQY * NP) + pq;
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        T sacc = 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) sacc += T(MEM ? mSx[q * NP + i] : tbz.S[q][i]) * w[q];
        o[i * NQ * NQY] = sacc;
      }
    }
    __syncthreads();
    sweep_c<1, NQ, NQY, NP, NP, true, false, Sy, 256, MEM>(tB, NQ * NQY * NP, tA, NQ * NP * NP, T(1), 3, 0, mSy);
    __syncthreads();
    sweep_c<0, NQ, NP, NP, NP, true, false, Sx, 256, MEM>(tA, NQ * NP * NP, s_r, NP3, T(1), 3, 0, mSx);
    __syncthreads();
  }

  // faces: neighbour layers of all six faces (one phase), then each direction
  T* s_nl = s_big;
  T* s_face = s_big + Sh::NL;
  {
    // neighbours across y = 0 and y = 1 (wrapped; unused on walls)
    const int y0 = ey == 0 ? M.ny - 1 : ey - 1, y1 = ey + 1 == M.ny ? 0 : ey + 1;
    nb_store<T, NP, NQ, CURVED, LE>(M, nbl, s_nl, s_nut, ex, ey, ez, ix, iz, T(M.ihy[y0]), T(M.ihy[y1]));
  }
  __syncthreads();
  if (CURVED)
    vel_faces_dir_curved<T, NP, NQ, NQY, ENR, 0>(M, e, s_u, s_nl, s_nut, s_r, s_face, s_ut, s_tab, ex, ey, ez, enr,
                                                 rt);
  else
    vel_faces_dir<T, NP, NQ, NQY, ENR, 0, MS, LE>(M, s_u, s_nl, s_nut, s_r, s_face, s_ut, ex, ey, ez, enr, hx, hy, hz, ix, iy,
                                           iz, rt);
  if (CURVED)
    vel_faces_dir_curved<T, NP, NQ, NQY, ENR, 1>(M, e, s_u, s_nl, s_nut, s_r, s_face, s_ut, s_tab, ex, ey, ez, enr,
                                                 rt);
  else
    vel_faces_dir<T, NP, NQ, NQY, ENR, 1, MS, LE>(M, s_u, s_nl, s_nut, s_r, s_face, s_ut, ex, ey, ez, enr, hx, hy, hz, ix, iy,
                                           iz, rt);
  if (CURVED)
    vel_faces_dir_curved<T, NP, NQ, NQY, ENR, 2>(M, e, s_u, s_nl, s_nut, s_r, s_face, s_ut, s_tab, ex, ey, ez, enr,
                                                 rt);
  else
    vel_faces_dir<T, NP, NQ, NQY, ENR, 2, MS, LE>(M, s_u, s_nl, s_nut, s_r, s_face, s_ut, ex, ey, ez, enr, hx, hy, hz, ix, iy,
                                           iz, rt);

  for (int i = tid; i < 3 * NP3; i += nt) r[e * 3 * NP3 + i] = s_r[i];
  if constexpr (ENR && LE == 1) {
    block_sum3(rt, s_red);
    if (tid < 3) r[M.enr_off + enr * 3 + tid] = rt[0];
  }
  if constexpr (ENR && LE != 1) {
    block_sum_n<3 * LE>(rt, s_red);
    if (tid < 3 * LE) r[M.enr_off + enr * 3 * LE + tid] = rt[0];
  }
}

// FP32 affine cells take the folded-face path (vel_cell below).
template <typename T>
__host__ __device__ constexpr bool vel_use_affine() { return sizeof(T) == 4; }

// Workgroups per CU the launch bounds plan for: the folded-face path is
// limited by its LDS, the general path by registers.
// (FP64 enriched cells keep up to 256 registers, other FP64 cells 168, FP32
// cells 128: below that they spill.)
template <typename T, int NP, int NQ, int NQY, bool ENR, bool CURVED, int LE = 1>
__host__ __device__ constexpr int vel_wg_per_cu() {
  if (CURVED) return 2;
  if (LE != 1) return ENR ? 2 : 3;  // general path; enriched cells hold 24 test-row sums
  if (!vel_use_affine<T>() || !AffShape<T, NP, NQ, NQY>::fits) return 3;
  const int by_lds = (160 * 1024) / AffShape<T, NP, NQ, NQY>::BYTES;
  const int by_regs = sizeof(T) == 8 ? (ENR ? 2 : 3) : 4;
  return by_lds < by_regs ? by_lds : by_regs;
}

// FP32 affine cells take the folded-face path (814 us against 1009 us for
// the general one on the 64x32x32 k = 4 mesh).  In FP64 that path reads one
// 8-byte LDS value per FMA in its extrapolations and lost to the general
// path's line-owned face phases (1516 us against 1430 us), so FP64, curved
// cells and the largest degrees take the general path.
// (degree-1 enrichment weights, LE = 8, always take the general path)
template <typename T, int NP, int NQ, int NQY, bool ENR, bool CURVED, int LE = 1>
__device__ __forceinline__ void vel_cell(const MeshDev& M, const T* __restrict__ u, T* __restrict__ r, int b,
                                         int layer_lo, int nlayers) {
  if constexpr (!CURVED && LE == 1 && vel_use_affine<T>() && AffShape<T, NP, NQ, NQY>::fits)
    vel_cell_affine<T, NP, NQ, NQY, ENR>(M, u, r, b, layer_lo, nlayers);
  else
    vel_cell_general<T, NP, NQ, NQY, ENR, CURVED, false, LE>(M, u, r, b, layer_lo, nlayers);
}

template <typename T, int NP, int NQ, int NQY, bool ENR, bool CURVED, int LE = 1>
__global__ __launch_bounds__(256, (vel_wg_per_cu<T, NP, NQ, NQY, ENR, CURVED, LE>())) void vel_kernel(const MeshDev M, const T* __restrict__ u, T* __restrict__ r,
                                                  int layer_lo, int nlayers) {
  // contiguous cell ranges per XCD (workgroups are dealt round-robin over
  // the 8 XCDs), so neighbouring cells share an L2
  const int nb = gridDim.x, bid = blockIdx.x;
  const int q8 = nb >> 3, r8 = nb & 7, xcd = bid & 7, m8 = bid >> 3;
  const int blk = xcd * q8 + (xcd < r8 ? xcd : r8) + m8;
  vel_cell<T, NP, NQ, NQY, ENR, CURVED, LE>(M, u, r, blk, layer_lo, nlayers);
}

}  // namespace

// Multiscale viscous operator (FP64, flat cells): the general cell path in
// its viscous-only mode.
template <int NP, int NQ, int NQY, bool ENR, int LE = 1>
__global__ __launch_bounds__(256, (LE == 8 && ENR) ? 2 : 3) void visc_ms_kernel(const MeshDev M, const double* __restrict__ u,
                                                         double* __restrict__ r, int layer_lo, int nlayers) {
  const int nb = gridDim.x, bid = blockIdx.x;
  const int q8 = nb >> 3, r8 = nb & 7, xcd = bid & 7, m8 = bid >> 3;
  const int blk = xcd * q8 + (xcd < r8 ? xcd : r8) + m8;
  vel_cell_general<double, NP, NQ, NQY, ENR, false, true, LE>(M, u, r, blk, layer_lo, nlayers);
}

// One mesh of a batched launch.
struct VelBatchItem {
  MeshDev M;
  const void* u;
  void* r;
  int layer_lo, nlayers;
};

namespace {

// Cells of many meshes (same degree and rules) in one launch: block b takes
// cell b of the concatenated cell ranges; prefix[i] is the first block of
// item i.  Each cell runs exactly the code of the single-mesh kernel, so the
// results are bit-for-bit the same.
template <typename T, int NP, int NQ, int NQY, bool ENR, bool CURVED>
__global__ __launch_bounds__(256, (vel_wg_per_cu<T, NP, NQ, NQY, ENR, CURVED>())) void vel_kernel_batched(const VelBatchItem* __restrict__ items,
                                                          const int64_t* __restrict__ prefix, int nitems) {
  const int64_t b = blockIdx.x;
  int lo = 0, hi = nitems;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= b) lo = mid; else hi = mid;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  const VelBatchItem& it = items[lo];
  vel_cell<T, NP, NQ, NQY, ENR, CURVED>(it.M, static_cast<const T*>(it.u), static_cast<T*>(it.r),
                                        (int)(b - prefix[lo]), it.layer_lo, it.nlayers);
}

template <typename T, int NP, int NQ, int NQW>
int launch_vel_t(const dg_mesh* m, const MeshDev& M, const void* u, void* r, hipStream_t s) {
  const T* uu = static_cast<const T*>(u);
  T* rr = static_cast<T*>(r);
  const int lo = (m->P.fully_periodic || m->lower_slot < 0) ? 0 : 1;
  const int hi = (m->P.fully_periodic || m->upper_slot < 0) ? m->P.ny - 1 : m->P.ny - 2;
  const int nl = hi - lo + 1;
  if (nl > 0) {
    const unsigned nb = (unsigned)((int64_t)m->P.nx * nl * m->P.nz);
    if (m->curved)
      hipLaunchKernelGGL((vel_kernel<T, NP, NQ, NQ, false, true>), dim3(nb), dim3(256), 0, s, M, uu, rr, lo, nl);
    else
      hipLaunchKernelGGL((vel_kernel<T, NP, NQ, NQ, false, false>), dim3(nb), dim3(256), 0, s, M, uu, rr, lo, nl);
  }
  if (m->nenr > 0) {
    if (m->curved)
      hipLaunchKernelGGL((vel_kernel<T, NP, NQ, NQW, true, true>), dim3((unsigned)m->nenr), dim3(256), 0, s, M, uu,
                         rr, 0, 0);
    else
      hipLaunchKernelGGL((vel_kernel<T, NP, NQ, NQW, true, false>), dim3((unsigned)m->nenr), dim3(256), 0, s, M,
                         uu, rr, 0, 0);
  }
  return check_hip(hipGetLastError(), "velocity kernel launch");
}

// Degree-1 enrichment weights (flat meshes): the regular cells' kernel reads
// the neighbours' 24 coefficients across the interface faces.
template <typename T, int NP, int NQ, int NQW>
int launch_vel_l1_t(const dg_mesh* m, const MeshDev& M, const void* u, void* r, hipStream_t s) {
  const T* uu = static_cast<const T*>(u);
  T* rr = static_cast<T*>(r);
  const int lo = (m->P.fully_periodic || m->lower_slot < 0) ? 0 : 1;
  const int hi = (m->P.fully_periodic || m->upper_slot < 0) ? m->P.ny - 1 : m->P.ny - 2;
  const int nl = hi - lo + 1;
  if (nl > 0) {
    const unsigned nb = (unsigned)((int64_t)m->P.nx * nl * m->P.nz);
    hipLaunchKernelGGL((vel_kernel<T, NP, NQ, NQ, false, false, 8>), dim3(nb), dim3(256), 0, s, M, uu, rr, lo, nl);
  }
  if (m->nenr > 0)
    hipLaunchKernelGGL((vel_kernel<T, NP, NQ, NQW, true, false, 8>), dim3((unsigned)m->nenr), dim3(256), 0, s, M, uu,
                       rr, 0, 0);
  return check_hip(hipGetLastError(), "velocity kernel launch");
}

MeshDev make_meshdev_u(const dg_mesh* m) {
  MeshDev M{};
  M.nx = m->P.nx;
  M.ny = m->P.ny;
  M.nz = m->P.nz;
  M.fully_periodic = m->P.fully_periodic;
  M.lower_slot = m->lower_slot;
  M.upper_slot = m->upper_slot;
  M.nslots = m->n_enr_layers;
  M.hx = m->hx;
  M.hz = m->hz;
  M.hy = m->hy;
  M.ihy = m->hy + m->P.ny;
  M.ihx = 1.0 / m->hx;
  M.ihz = 1.0 / m->hz;
  M.tab = m->tab_u;
  M.psi = m->psi;
  M.psi_pts = m->psi_pts;
  for (int f = 0; f <= 6; ++f) M.psi_off[f] = (f == 0) ? 0 : psi_face_offset(m->P.nq_u, m->P.nq_wn, f - 1);
  M.nu = m->P.nu;
  M.theta = m->P.theta;
  M.pen = m->P.ip_factor_u * (m->P.k_u + 1.0) * (m->P.k_u + 1.0);
  M.wall_mult = m->P.wall_ip_mult;
  M.enr_off = m->ncell * 3 * (int64_t)m->np_u * m->np_u * m->np_u;
  M.geo = m->geo;
  M.geo_stride = m->geo_stride;
  M.tauF = m->tauF;
  M.nq_wn = m->P.nq_wn;
  M.nut = nullptr;
  return M;
}

}  // namespace

// (np, nq, nq_wn) combinations compiled in.
#define DG_VEL_COMBOS(X) \
  X(3, 4, 8)             \
  X(3, 4, 4)             \
  X(4, 4, 8)             \
  X(4, 5, 8)             \
  X(4, 5, 5)             \
  X(5, 7, 8)             \
  X(6, 8, 8)

// (np, nq, nq_wn) combinations compiled in for degree-1 enrichment weights.
#define DG_VEL_L1_COMBOS(X) \
  X(3, 4, 8)                \
  X(4, 4, 8)                \
  X(4, 5, 8)                \
  X(5, 7, 8)

// Regular-layer range of a mesh (cells not in an enriched layer).
static void regular_layers(const dg_mesh* m, int& lo, int& nl) {
  lo = (m->P.fully_periodic || m->lower_slot < 0) ? 0 : 1;
  const int hi = (m->P.fully_periodic || m->upper_slot < 0) ? m->P.ny - 1 : m->P.ny - 2;
  nl = hi - lo + 1;
}

template <typename T, int NP, int NQ, int NQW, bool CURVED>
static void launch_batch_group(const VelBatchItem* d_items_reg, const int64_t* d_pre_reg, int nreg, int64_t tot_reg,
                               const VelBatchItem* d_items_enr, const int64_t* d_pre_enr, int nenr, int64_t tot_enr,
                               hipStream_t s) {
  if (nreg > 0 && tot_reg > 0)
    hipLaunchKernelGGL((vel_kernel_batched<T, NP, NQ, NQ, false, CURVED>), dim3((unsigned)tot_reg), dim3(256), 0, s,
                       d_items_reg, d_pre_reg, nreg);
  if (nenr > 0 && tot_enr > 0)
    hipLaunchKernelGGL((vel_kernel_batched<T, NP, NQ, NQW, true, CURVED>), dim3((unsigned)tot_enr), dim3(256), 0, s,
                       d_items_enr, d_pre_enr, nenr);
}

bool velocity_supported(int np, int nq, int nqy) {
#define X(a, b, c) \
  if (np == a && nq == b && nqy == c) return true;
  DG_VEL_COMBOS(X)
#undef X
  return false;
}

const char* velocity_combos() { return "velocity (k+1, nq_u, nq_wn): (3,4,8) (3,4,4) (4,4,8) (4,5,8) (4,5,5) (5,7,8) (6,8,8)"; }

bool velocity_l1_supported(int np, int nq, int nqy) {
#define X(a, b, c) \
  if (np == a && nq == b && nqy == c) return true;
  DG_VEL_L1_COMBOS(X)
#undef X
  return false;
}

const char* velocity_l1_combos() { return "(3,4,8) (4,4,8) (4,5,8) (5,7,8)"; }

template <int NP, int NQ, int NQW>
static int launch_visc_ms_t(const dg_mesh* m, MeshDev M, const double* u, double* r, hipStream_t s) {
  const int lo = (m->P.fully_periodic || m->lower_slot < 0) ? 0 : 1;
  const int hi = (m->P.fully_periodic || m->upper_slot < 0) ? m->P.ny - 1 : m->P.ny - 2;
  const int nl = hi - lo + 1;
  if (nl > 0)
    hipLaunchKernelGGL((visc_ms_kernel<NP, NQ, NQ, false>), dim3((unsigned)((int64_t)m->P.nx * nl * m->P.nz)),
                       dim3(256), 0, s, M, u, r, lo, nl);
  if (m->nenr > 0)
    hipLaunchKernelGGL((visc_ms_kernel<NP, NQ, NQW, true>), dim3((unsigned)m->nenr), dim3(256), 0, s, M, u, r, 0, 0);
  return check_hip(hipGetLastError(), "multiscale viscous kernel launch");
}

// Degree-1 enrichment weights: the regular cells read the 24 coefficients of
// an enriched neighbour.
template <int NP, int NQ, int NQW>
static int launch_visc_ms_l1_t(const dg_mesh* m, MeshDev M, const double* u, double* r, hipStream_t s) {
  const int lo = (m->P.fully_periodic || m->lower_slot < 0) ? 0 : 1;
  const int hi = (m->P.fully_periodic || m->upper_slot < 0) ? m->P.ny - 1 : m->P.ny - 2;
  const int nl = hi - lo + 1;
  if (nl > 0)
    hipLaunchKernelGGL((visc_ms_kernel<NP, NQ, NQ, false, 8>), dim3((unsigned)((int64_t)m->P.nx * nl * m->P.nz)),
                       dim3(256), 0, s, M, u, r, lo, nl);
  hipLaunchKernelGGL((visc_ms_kernel<NP, NQ, NQW, true, 8>), dim3((unsigned)m->nenr), dim3(256), 0, s, M, u, r, 0, 0);
  return check_hip(hipGetLastError(), "multiscale viscous kernel launch");
}

int launch_viscous_multiscale(const dg_mesh* m, const double* nut, const double* u, double* out, hipStream_t s) {
  MeshDev M = make_meshdev_u(m);
  M.nut = nut;
  const int np = m->np_u, nq = m->P.nq_u, nqw = m->P.nq_wn;
  if (m->nle != 1 && m->nenr > 0) {
#define X(a, b, c) \
  if (np == a && nq == b && nqw == c) return launch_visc_ms_l1_t<a, b, c>(m, M, u, out, s);
    DG_VEL_L1_COMBOS(X)
#undef X
    return set_error(DG_ERR_UNSUPPORTED, "degree-1 enrichment weights: combination not compiled");
  }
#define X(a, b, c)                                                        \
  if (np == a && nq == b && (nqw == c || m->nenr == 0)) return launch_visc_ms_t<a, b, c>(m, M, u, out, s);
  DG_VEL_COMBOS(X)
#undef X
  return set_error(DG_ERR_UNSUPPORTED, "velocity degree/quadrature combination not compiled");
}

int launch_velocity(const dg_mesh* m, dg_prec prec, const void* u, void* r, hipStream_t s, bool convective_only) {
  MeshDev M = make_meshdev_u(m);
  if (convective_only) M.nu = 0.0;  // every viscous term carries a factor nu
  const int np = m->np_u, nq = m->P.nq_u, nqw = m->P.nq_wn;
  if (m->nle != 1 && m->nenr > 0) {
#define X(a, b, c)                                                                 \
  if (np == a && nq == b && nqw == c) {                                            \
    return prec == DG_F64 ? launch_vel_l1_t<double, a, b, c>(m, M, u, r, s)        \
                          : launch_vel_l1_t<float, a, b, c>(m, M, u, r, s);        \
  }
    DG_VEL_L1_COMBOS(X)
#undef X
    return set_error(DG_ERR_UNSUPPORTED, std::string("degree-1 enrichment weights: (k_u+1, nq_u, nq_wn) not "
                                                     "compiled; have ") + velocity_l1_combos());
  }
  // without enriched cells only the regular kernel runs: nq_wn is irrelevant
#define X(a, b, c)                                                                 \
  if (np == a && nq == b && (nqw == c || m->nenr == 0)) {                          \
    return prec == DG_F64 ? launch_vel_t<double, a, b, c>(m, M, u, r, s)           \
                          : launch_vel_t<float, a, b, c>(m, M, u, r, s);           \
  }
  DG_VEL_COMBOS(X)
#undef X
  return set_error(DG_ERR_UNSUPPORTED, "velocity degree/quadrature combination not compiled");
}

}  // namespace dgwm

namespace dgwm {

// At most two descriptors per mesh (regular and enriched cells) and, per
// group and class, one prefix entry per descriptor plus the total.
int64_t batch_workspace_bytes(int n) {
  const size_t items = ((2 * (size_t)n * sizeof(VelBatchItem)) + 255) & ~size_t(255);
  return (int64_t)(items + (4 * (size_t)n + 2) * sizeof(int64_t));
}

// Groups the meshes by compiled combination and launches one batched kernel
// per group and cell class (regular / enriched).
namespace {

// Pinned staging ring of the batched call, per host thread: each call
// takes the next slot, first waiting for the copy that last used it (long
// done unless kStageSlots calls are still queued), and marks its own copy
// with the slot's event.
constexpr int kStageSlots = 8;
struct StageRing {
  char* p[kStageSlots] = {};
  size_t cap[kStageSlots] = {};
  hipEvent_t ev[kStageSlots] = {};
  bool used[kStageSlots] = {};
  int next = 0, cur = -1;
};
thread_local StageRing tl_ring;

int stage_slot(size_t bytes, char** out) {
  StageRing& R = tl_ring;
  const int k = R.next;
  R.next = (k + 1) % kStageSlots;
  if (!R.ev[k] && hipEventCreateWithFlags(&R.ev[k], hipEventDisableTiming) != hipSuccess)
    return set_error(DG_ERR_HIP, "staging event creation failed");
  if (R.used[k])
    if (int rc = check_hip(hipEventSynchronize(R.ev[k]), "staging slot reuse")) return rc;
  if (R.cap[k] < bytes) {
    if (R.p[k]) (void)hipHostFree(R.p[k]);
    R.p[k] = nullptr;
    R.cap[k] = 0;
    void* q = nullptr;
    const size_t want = std::max<size_t>(bytes, 64 << 10);
    if (int rc = check_hip(hipHostMalloc(&q, want, hipHostMallocDefault), "pinned staging")) return rc;
    R.p[k] = static_cast<char*>(q);
    R.cap[k] = want;
  }
  R.cur = k;
  *out = R.p[k];
  return DG_OK;
}

int stage_release(hipStream_t s) {
  StageRing& R = tl_ring;
  R.used[R.cur] = true;
  return check_hip(hipEventRecord(R.ev[R.cur], s), "staging event");
}

}  // namespace

int launch_velocity_batched(const dg_mesh* const* meshes, int n, dg_prec prec, const void* const* u, void* const* r,
                            void* ws, size_t ws_bytes, hipStream_t s) {
  if ((int64_t)ws_bytes < batch_workspace_bytes(n)) return set_error(DG_ERR_WORKSPACE, "batch workspace too small");
  struct Key {
    int np, nq, nqw, curved;
    bool operator==(const Key& o) const { return np == o.np && nq == o.nq && nqw == o.nqw && curved == o.curved; }
  };
  std::vector<Key> keys;
  std::vector<int> key_of(n);
  for (int i = 0; i < n; ++i) {
    const dg_mesh* m = meshes[i];
    Key k{m->np_u, m->P.nq_u, m->nenr > 0 ? m->P.nq_wn : -1, m->curved};
    int j = 0;
    for (; j < (int)keys.size(); ++j)
      if (keys[j] == k) break;
    if (j == (int)keys.size()) keys.push_back(k);
    key_of[i] = j;
  }
  // host staging: per group, regular items then enriched items, with prefixes
  std::vector<VelBatchItem> items;
  std::vector<int64_t> pre;
  struct Group { int ireg, nreg, preg, ienr, nenr, penr; int64_t treg, tenr; Key k; };
  std::vector<Group> groups;
  for (int g = 0; g < (int)keys.size(); ++g) {
    Group G{};
    G.k = keys[g];
    for (int cls = 0; cls < 2; ++cls) {
      const int first = (int)items.size(), pfirst = (int)pre.size();
      int64_t tot = 0;
      for (int i = 0; i < n; ++i) {
        if (key_of[i] != g) continue;
        const dg_mesh* m = meshes[i];
        int lo, nl;
        regular_layers(m, lo, nl);
        const int64_t nb = cls == 0 ? (nl > 0 ? (int64_t)m->P.nx * nl * m->P.nz : 0) : m->nenr;
        if (nb == 0) continue;
        VelBatchItem it{};
        it.M = make_meshdev_u(m);
        it.u = u[i];
        it.r = r[i];
        it.layer_lo = lo;
        it.nlayers = nl;
        items.push_back(it);
        pre.push_back(tot);
        tot += nb;
      }
      pre.push_back(tot);
      if (cls == 0) { G.ireg = first; G.nreg = (int)items.size() - first; G.preg = pfirst; G.treg = tot; }
      else { G.ienr = first; G.nenr = (int)items.size() - first; G.penr = pfirst; G.tenr = tot; }
    }
    groups.push_back(G);
  }
  char* base = static_cast<char*>(ws);
  const size_t items_bytes = (items.size() * sizeof(VelBatchItem) + 255) & ~size_t(255);
  VelBatchItem* d_items = reinterpret_cast<VelBatchItem*>(base);
  int64_t* d_pre = reinterpret_cast<int64_t*>(base + items_bytes);
  // descriptors and prefixes go up in one copy from a pinned staging slot
  // (no host wait: the slot is reused only after its copy has run)
  char* stage = nullptr;
  int rc = stage_slot(items_bytes + pre.size() * sizeof(int64_t), &stage);
  if (rc) return rc;
  if (!items.empty()) std::memcpy(stage, items.data(), items.size() * sizeof(VelBatchItem));
  std::memcpy(stage + items_bytes, pre.data(), pre.size() * sizeof(int64_t));
  rc = check_hip(hipMemcpyAsync(base, stage, items_bytes + pre.size() * sizeof(int64_t), hipMemcpyHostToDevice, s),
                 "batch descriptors");
  if (!rc) rc = stage_release(s);
  if (rc) return rc;
  for (const Group& G : groups) {
    bool done = false;
#define X(a, b, c)                                                                                               \
  if (!done && G.k.np == a && G.k.nq == b && (G.k.nqw == c || G.k.nqw < 0)) {                                    \
    done = true;                                                                                                 \
    if (prec == DG_F64) {                                                                                        \
      if (G.k.curved)                                                                                            \
        launch_batch_group<double, a, b, c, true>(d_items + G.ireg, d_pre + G.preg, G.nreg, G.treg,              \
                                                  d_items + G.ienr, d_pre + G.penr, G.nenr, G.tenr, s);          \
      else                                                                                                       \
        launch_batch_group<double, a, b, c, false>(d_items + G.ireg, d_pre + G.preg, G.nreg, G.treg,             \
                                                   d_items + G.ienr, d_pre + G.penr, G.nenr, G.tenr, s);         \
    } else {                                                                                                     \
      if (G.k.curved)                                                                                            \
        launch_batch_group<float, a, b, c, true>(d_items + G.ireg, d_pre + G.preg, G.nreg, G.treg,               \
                                                 d_items + G.ienr, d_pre + G.penr, G.nenr, G.tenr, s);           \
      else                                                                                                       \
        launch_batch_group<float, a, b, c, false>(d_items + G.ireg, d_pre + G.preg, G.nreg, G.treg,              \
                                                  d_items + G.ienr, d_pre + G.penr, G.nenr, G.tenr, s);          \
    }                                                                                                            \
  }
    DG_VEL_COMBOS(X)
#undef X
    if (!done) return set_error(DG_ERR_UNSUPPORTED, "velocity combination not compiled");
  }
  return check_hip(hipGetLastError(), "batched velocity launch");
}

}  // namespace dgwm
