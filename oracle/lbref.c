/*
 * FP64 CPU oracle for the regularized lattice Boltzmann step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may use it.  It shares no code, header, table or
 * constant with the GPU path.
 *
 * What it computes (Montessori et al., "Thread-safe lattice Boltzmann for
 * high-performance computing on GPUs"):
 *
 *   The thread-safe method of Section 3 changes only *where* a post-collision
 *   population is evaluated (at the destination, from the neighbour's
 *   moments) and not *what* is evaluated.  Its result is therefore exactly
 *   the result of a conventional regularized BGK step: collide every node,
 *   then stream every post-collision population to its neighbour.  This file
 *   writes that conventional step out literally, with two population arrays
 *   and push streaming:
 *
 *   1. moments (Section 2, moment definitions; Section 4, moment snippet):
 *        rho = sum_a f_a,  j = sum_a f_a c_a,
 *        u   = (j + F/2) / rho0                      (incompressible model,
 *                                                     half-force shift)
 *   2. equilibrium (Section 2, eq. equil, He-Luo incompressible form):
 *        f^eq_a = t_a [ rho + rho0 ( c.u/cs2 + H2_a:uu/(2 cs4) ) ]
 *        (order 3 adds rho0 H3_a:uuu/(6 cs6), the next term of the same
 *        Hermite series, eq. hermite)
 *   3. non-equilibrium and its Hermite projection (Section 3, eq. hermite):
 *        f^neq_a = f_a - f^eq_a
 *        a1 = sum_a f^neq_a c_a,  Pi = sum_a f^neq_a c_a c_a
 *        fhat_a = t_a [ c.a1/cs2 + H2_a:Pi/(2 cs4) (+ H3_a:a3/(6 cs6)) ]
 *        with a3 = u Pi + perms (recursive third-order coefficient).
 *        Without a body force a1 vanishes and this is the compact second-order
 *        formula of Section 3.
 *   4. post-collision (Section 3, eq. LBexp) plus Guo's body-force source:
 *        f^pc_a = f^eq_a + (1 - omega) fhat_a + (1 - omega/2) S_a,
 *        S_a = t_a [ (c_a - u).F/cs2 + (c_a.u)(c_a.F)/cs4 ]
 *   5. streaming (Section 2, eq. lbe; Section 3, eq. pushLB):
 *        f_a(x + c_a) <- f^pc_a(x), periodic wrap per axis, or halfway
 *        bounce-back f_{abar}(x) <- f^pc_a(x) when x + c_a leaves the
 *        domain across a wall.
 *   6. moving walls (Section 5, lid-driven cavity, where the lid's motion
 *        enters through Bouzidi's momentum correction; at the halfway
 *        position that correction is Ladd's):
 *        f_{abar}(x) <- f^pc_a(x) - 2 t_a rho0 (c_a . u_w) / cs2,
 *        with u_w the velocity of the wall that x + c_a crosses; a link that
 *        leaves across an edge or corner takes the sum over the walls it
 *        crosses.  rho0 is the wall density of the incompressible model.
 *
 *   Lattices: textbook D2Q9, D3Q19, D3Q27 with cs2 = 1/3 (the paper cites but
 *   does not print the weights).
 *
 *   Two-species colour-gradient collision (Section 2.1) is in
 *   step_two_species below, with the near-contact interactions of Section
 *   2.2 (nci_flags, nci_force).
 *
 * Compiled with -ffp-contract=off so that every node performs bit-identical
 * arithmetic (translation equivariance is a test).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Domains below this many nodes run their node loops on one thread: the
 * per-step fork/join of a parallel loop costs more than the work there.  Each
 * node's arithmetic is independent of the thread count. */
#define OMP_MIN_NODES 16384

#define CS2 (1.0 / 3.0)
#define CS4 (CS2 * CS2)
#define CS6 (CS4 * CS2)

typedef struct {
  int32_t lattice;  /* 9 = D2Q9, 19 = D3Q19, 27 = D3Q27 */
  int32_t order;    /* 2 or 3: Hermite order of equilibrium and regularization */
  int64_t nx, ny, nz;
  int32_t bb[3];    /* per axis: 0 periodic, 1 halfway bounce-back walls at both ends */
  int32_t species;  /* 1 or 2 */
  double tau;       /* relaxation time, omega = 1/tau */
  double rho0;      /* bulk density of the incompressible equilibrium */
  double force[3];  /* body-force density */
  double sigma;     /* colour-gradient surface tension parameter */
  double beta;      /* recolouring (anti-diffusion) parameter */
  double wall_u[3][2][3]; /* velocity of the wall at [axis][low, high]: tangential,
                             bounce-back axes only, one species only */
  double nci_strength;    /* near-contact force constant A (two species); 0 = off */
  double nci_eps;         /* bulk threshold: a node is bulk if phi < -1 + eps */
  int32_t nci_reach;      /* sampling distance d along a lattice direction (>= 1) */
  int32_t pad_;
} ref_params;

typedef struct {
  int q, d;
  int c[27][3];
  double w[27];
  int opp[27];
  double h2[27][3][3];     /* H2_a = c c - cs2 I */
  double h3[27][3][3][3];  /* H3_a = c c c - cs2 (c I + perms) */
} lattice_t;

/* Textbook velocity sets: every c in {-1,0,1}^D up to a maximum |c|^2, with
 * weights that depend on |c|^2 only. */
static int build_lattice(int kind, lattice_t* L) {
  double wc2[4];
  int d, maxc2;
  if (kind == 9) {
    d = 2; maxc2 = 2;
    wc2[0] = 4.0 / 9.0; wc2[1] = 1.0 / 9.0; wc2[2] = 1.0 / 36.0; wc2[3] = 0.0;
  } else if (kind == 19) {
    d = 3; maxc2 = 2;
    wc2[0] = 1.0 / 3.0; wc2[1] = 1.0 / 18.0; wc2[2] = 1.0 / 36.0; wc2[3] = 0.0;
  } else if (kind == 27) {
    d = 3; maxc2 = 3;
    wc2[0] = 8.0 / 27.0; wc2[1] = 2.0 / 27.0; wc2[2] = 1.0 / 54.0; wc2[3] = 1.0 / 216.0;
  } else {
    return -1;
  }
  memset(L, 0, sizeof(*L));
  L->d = d;
  int q = 0;
  int zlo = (d == 3) ? -1 : 0, zhi = (d == 3) ? 1 : 0;
  for (int cz = zlo; cz <= zhi; ++cz)
    for (int cy = -1; cy <= 1; ++cy)
      for (int cx = -1; cx <= 1; ++cx) {
        int c2 = cx * cx + cy * cy + cz * cz;
        if (c2 > maxc2) continue;
        L->c[q][0] = cx; L->c[q][1] = cy; L->c[q][2] = cz;
        L->w[q] = wc2[c2];
        ++q;
      }
  L->q = q;
  for (int a = 0; a < q; ++a) {
    L->opp[a] = -1;
    for (int b = 0; b < q; ++b)
      if (L->c[b][0] == -L->c[a][0] && L->c[b][1] == -L->c[a][1] && L->c[b][2] == -L->c[a][2])
        L->opp[a] = b;
    for (int al = 0; al < 3; ++al)
      for (int be = 0; be < 3; ++be) {
        L->h2[a][al][be] = (double)(L->c[a][al] * L->c[a][be]) - (al == be ? CS2 : 0.0);
        for (int ga = 0; ga < 3; ++ga) {
          double t = (double)(L->c[a][al] * L->c[a][be] * L->c[a][ga]);
          if (be == ga) t -= CS2 * L->c[a][al];
          if (al == ga) t -= CS2 * L->c[a][be];
          if (al == be) t -= CS2 * L->c[a][ga];
          L->h3[a][al][be][ga] = t;
        }
      }
  }
  return 0;
}

/* H2_a : X over the lattice dimensions. */
static double h2dot(const lattice_t* L, int a, const double X[3][3]) {
  double s = 0.0;
  for (int al = 0; al < L->d; ++al)
    for (int be = 0; be < L->d; ++be) s += L->h2[a][al][be] * X[al][be];
  return s;
}

/* H3_a : X over the lattice dimensions (full rank-3 contraction). */
static double h3dot(const lattice_t* L, int a, const double X[3][3][3]) {
  double s = 0.0;
  for (int al = 0; al < L->d; ++al)
    for (int be = 0; be < L->d; ++be)
      for (int ga = 0; ga < L->d; ++ga) s += L->h3[a][al][be][ga] * X[al][be][ga];
  return s;
}

static double cdot(const lattice_t* L, int a, const double v[3]) {
  double s = 0.0;
  for (int al = 0; al < L->d; ++al) s += L->c[a][al] * v[al];
  return s;
}

/* Incompressible equilibrium (eq. equil), optionally extended to the
 * third-order Hermite term. */
static void equilibrium(const lattice_t* L, const ref_params* p, double rho, const double u[3],
                        double* feq) {
  double uu[3][3], uuu[3][3][3];
  for (int al = 0; al < 3; ++al)
    for (int be = 0; be < 3; ++be) {
      uu[al][be] = u[al] * u[be];
      for (int ga = 0; ga < 3; ++ga) uuu[al][be][ga] = u[al] * u[be] * u[ga];
    }
  for (int a = 0; a < L->q; ++a) {
    double e = cdot(L, a, u) / CS2 + h2dot(L, a, uu) / (2.0 * CS4);
    if (p->order >= 3) e += h3dot(L, a, uuu) / (6.0 * CS6);
    feq[a] = L->w[a] * (rho + p->rho0 * e);
  }
}

/* Moments of one node: rho, j, and the velocity of the forced incompressible
 * model u = (j + F/2)/rho0 for the body force F acting on the node. */
static void node_moments_f(const lattice_t* L, const ref_params* p, const double* f,
                           const double F[3], double* rho, double j[3], double u[3]) {
  double r = 0.0;
  j[0] = j[1] = j[2] = 0.0;
  for (int a = 0; a < L->q; ++a) {
    r += f[a];
    for (int al = 0; al < 3; ++al) j[al] += f[a] * L->c[a][al];
  }
  *rho = r;
  for (int al = 0; al < 3; ++al) u[al] = (j[al] + 0.5 * F[al]) / p->rho0;
}

static void node_moments(const lattice_t* L, const ref_params* p, const double* f, double* rho,
                         double j[3], double u[3]) {
  node_moments_f(L, p, f, p->force, rho, j, u);
}

/* Regularized collision of one node under the body force F: f (Q values) ->
 * f^pc (Q values).  Steps 1-4 of the header. */
static void collide_f(const lattice_t* L, const ref_params* p, const double* f,
                      const double F[3], double* fpc) {
  const int Q = L->q;
  const double omega = 1.0 / p->tau;
  double rho, j[3], u[3];
  node_moments_f(L, p, f, F, &rho, j, u);

  double feq[27], fneq[27];
  equilibrium(L, p, rho, u, feq);
  for (int a = 0; a < Q; ++a) fneq[a] = f[a] - feq[a];

  double a1[3] = {0.0, 0.0, 0.0};
  double Pi[3][3] = {{0.0}};
  for (int a = 0; a < Q; ++a)
    for (int al = 0; al < 3; ++al) {
      a1[al] += fneq[a] * L->c[a][al];
      for (int be = 0; be < 3; ++be) Pi[al][be] += fneq[a] * L->c[a][al] * L->c[a][be];
    }
  double a3[3][3][3];
  for (int al = 0; al < 3; ++al)
    for (int be = 0; be < 3; ++be)
      for (int ga = 0; ga < 3; ++ga)
        a3[al][be][ga] = u[al] * Pi[be][ga] + u[be] * Pi[al][ga] + u[ga] * Pi[al][be];

  for (int a = 0; a < Q; ++a) {
    double fhat = cdot(L, a, a1) / CS2 + h2dot(L, a, Pi) / (2.0 * CS4);
    if (p->order >= 3) fhat += h3dot(L, a, a3) / (6.0 * CS6);
    fhat *= L->w[a];
    /* Guo, Zheng & Shi (2002) source, written in its published form. */
    double cmuF = 0.0;
    for (int al = 0; al < L->d; ++al) cmuF += (L->c[a][al] - u[al]) * F[al];
    double S = L->w[a] * (cmuF / CS2 + cdot(L, a, u) * cdot(L, a, F) / CS4);
    fpc[a] = feq[a] + (1.0 - omega) * fhat + (1.0 - 0.5 * omega) * S;
  }
}

/* Collision under the problem's constant body force. */
static void collide(const lattice_t* L, const ref_params* p, const double* f, double* fpc) {
  collide_f(L, p, f, p->force, fpc);
}

/* Destination of population a leaving node (x,y,z).  Returns 1 and the linear
 * destination index when it stays in the domain (after periodic wrap), 0 when
 * it crosses a bounce-back wall. */
static int destination(const lattice_t* L, const ref_params* p, int a, int64_t x, int64_t y,
                       int64_t z, int64_t* dst) {
  int64_t n[3] = {p->nx, p->ny, p->nz};
  int64_t t[3] = {x + L->c[a][0], y + L->c[a][1], z + L->c[a][2]};
  for (int al = 0; al < 3; ++al) {
    if (t[al] < 0 || t[al] >= n[al]) {
      if (p->bb[al]) return 0;
      t[al] = (t[al] + n[al]) % n[al];
    }
  }
  *dst = t[0] + n[0] * (t[1] + n[1] * t[2]);
  return 1;
}

static int check_params(const ref_params* p, lattice_t* L) {
  if (build_lattice(p->lattice, L) != 0) return -1;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return -1;
  if (L->d == 2 && p->nz != 1) return -1;
  if (!(p->tau > 0.5)) return -1;
  if (p->order != 2 && p->order != 3) return -1;
  if (p->species != 1 && p->species != 2) return -1;
  if (p->nci_strength != 0.0 && (p->species != 2 || p->nci_reach < 1 || !(p->nci_eps > 0.0)))
    return -1;
  /* wall velocities: tangential, on bounce-back axes, one species */
  for (int al = 0; al < 3; ++al)
    for (int side = 0; side < 2; ++side)
      for (int be = 0; be < 3; ++be) {
        const double v = p->wall_u[al][side][be];
        if (v == 0.0) continue;
        if (!p->bb[al] || be == al || be >= L->d || p->species != 1) return -1;
      }
  return 0;
}

/* Momentum correction of a link a of node (x, y, z) that leaves the domain
 * across one or more walls: -2 t_a rho0 (c_a . sum of the crossed walls'
 * velocities) / cs2. */
static double wall_term(const lattice_t* L, const ref_params* p, int a, int64_t x, int64_t y,
                        int64_t z) {
  const int64_t n[3] = {p->nx, p->ny, p->nz};
  const int64_t t[3] = {x + L->c[a][0], y + L->c[a][1], z + L->c[a][2]};
  double cu = 0.0;
  for (int al = 0; al < 3; ++al) {
    if (!p->bb[al]) continue;
    int side = -1;
    if (t[al] < 0) side = 0;
    if (t[al] >= n[al]) side = 1;
    if (side < 0) continue;
    for (int be = 0; be < 3; ++be) cu += L->c[a][be] * p->wall_u[al][side][be];
  }
  return -2.0 * L->w[a] * p->rho0 * cu / CS2;
}

/* ------------------------------------------------------------------------ */
/* Two-species colour-gradient step (Section 2.1).                            */
/*                                                                            */
/*   g = f_R + f_B is relaxed with the regularized collision above (one set  */
/*   of moments for the mixture), perturbed by                               */
/*     Omega1_a = (9/4) sigma omega |G| ( t_a (c_a.G)^2/|G|^2 - B_a ),        */
/*   G = grad phi, phi = (rho_R - rho_B)/(rho_R + rho_B), and recoloured      */
/*     f_R,a = (rho_R/rho) g*_a + beta (rho_R rho_B/rho) t_a cos(theta_a)     */
/*     f_B,a = (rho_B/rho) g*_a - beta (rho_R rho_B/rho) t_a cos(theta_a)     */
/*   with cos(theta_a) = c_a.G/(|c_a||G|), before each species is streamed.   */
/*   grad phi uses the isotropic lattice stencil                              */
/*     grad phi(x) = (1/cs2) sum_b t_b c_b phi(x + c_b).                      */
/*   Where |G|^2 <= 1e-20 both the perturbation and cos(theta) are zero.      */
/* ------------------------------------------------------------------------ */

/* B_a weights for the colour-gradient perturbation (Liu, Valocchi & Kang
 * 2012; Reis & Phillips 2007 for D2Q9).  They satisfy sum_a B_a = cs2, so the
 * perturbation carries no mass:
 *   D2Q9 : B_0 = -4/27, B_{|c|^2=1} = 2/27, B_{|c|^2=2} = 5/108
 *   D3Q19: B_0 = -1/3,  B_{|c|^2=1} = 1/18, B_{|c|^2=2} = 1/36
 * (for D3Q19 these equal the lattice weights with the rest weight negated). */
static void weights_B(const lattice_t* L, double* B) {
  for (int a = 0; a < L->q; ++a) {
    int c2 = L->c[a][0] * L->c[a][0] + L->c[a][1] * L->c[a][1] + L->c[a][2] * L->c[a][2];
    if (L->q == 9) {
      B[a] = (c2 == 0) ? -4.0 / 27.0 : (c2 == 1 ? 2.0 / 27.0 : 5.0 / 108.0);
    } else {
      B[a] = (c2 == 0) ? -1.0 / 3.0 : (c2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
  }
}

static void phase_field(const lattice_t* L, const ref_params* p, const double* f, int64_t N,
                        double* phi) {
  const int Q = L->q;
  (void)p;
#pragma omp parallel for schedule(static) if (N >= OMP_MIN_NODES)
  for (int64_t n = 0; n < N; ++n) {
    double rr = 0.0, rb = 0.0;
    for (int a = 0; a < Q; ++a) {
      rr += f[(int64_t)a * N + n];
      rb += f[(int64_t)(Q + a) * N + n];
    }
    phi[n] = (rr - rb) / (rr + rb);
  }
}

/* Isotropic gradient of phi at node (x,y,z).  Neighbours beyond a
 * bounce-back wall take the value of the node itself (zero normal gradient). */
static void gradient(const lattice_t* L, const ref_params* p, const double* phi, int64_t x,
                     int64_t y, int64_t z, double G[3]) {
  int64_t n[3] = {p->nx, p->ny, p->nz};
  int64_t self = x + n[0] * (y + n[1] * z);
  G[0] = G[1] = G[2] = 0.0;
  for (int b = 0; b < L->q; ++b) {
    int64_t t[3] = {x + L->c[b][0], y + L->c[b][1], z + L->c[b][2]};
    int inside = 1;
    for (int al = 0; al < 3; ++al)
      if (t[al] < 0 || t[al] >= n[al]) {
        if (p->bb[al]) inside = 0;
        else t[al] = (t[al] + n[al]) % n[al];
      }
    double v = inside ? phi[t[0] + n[0] * (t[1] + n[1] * t[2])] : phi[self];
    for (int al = 0; al < 3; ++al) G[al] += L->w[b] * L->c[b][al] * v;
  }
  for (int al = 0; al < 3; ++al) G[al] /= CS2;
}

/* ------------------------------------------------------------------------ */
/* Near-contact interactions (Section 2.2).                                   */
/*                                                                            */
/*   Flagging pass, before the collision, in the paper's scatter form:       */
/*   sitting on a bulk node x of the continuous phase, phi(x) < -1 + eps,     */
/*   sample phi at the two points x + d c_a and x - d c_a of every pair of    */
/*   opposite lattice directions (d = nci_reach).  When neither point is      */
/*   bulk (both phi > -1 + eps), an interface lies on each side of x along    */
/*   c_a, and both points are flagged.  A point beyond a bounce-back wall is  */
/*   not sampled; periodic axes wrap.                                         */
/*   Force: a flagged node y whose phase gradient G is defined (|G|^2 >      */
/*   1e-20) carries F_nci(y) = A rho_R(y) G/|G|, along the interface normal   */
/*   into the dispersed phase (red, phi > 0: the droplets), proportional to   */
/*   the dispersed density at y.  In the collision it acts on the mixture     */
/*   like the constant body force (Guo source, half-force velocity shift).    */
/* ------------------------------------------------------------------------ */

/* Linear index of the point (x, y, z) + d c; 0 if it lies beyond a wall. */
static int sample_point(const ref_params* p, int64_t x, int64_t y, int64_t z, const int c[3],
                        int64_t d, int64_t* out) {
  const int64_t n[3] = {p->nx, p->ny, p->nz};
  int64_t t[3] = {x + d * c[0], y + d * c[1], z + d * c[2]};
  for (int al = 0; al < 3; ++al) {
    if (t[al] < 0 || t[al] >= n[al]) {
      if (p->bb[al]) return 0;
      t[al] = ((t[al] % n[al]) + n[al]) % n[al];
    }
  }
  *out = t[0] + n[0] * (t[1] + n[1] * t[2]);
  return 1;
}

static void nci_flags(const lattice_t* L, const ref_params* p, const double* phi,
                      unsigned char* flag) {
  const int64_t nx = p->nx, ny = p->ny, nz = p->nz;
  const int64_t N = nx * ny * nz;
  const double thr = -1.0 + p->nci_eps;
  const int64_t d = p->nci_reach;
  memset(flag, 0, (size_t)N);
  for (int64_t z = 0; z < nz; ++z)
    for (int64_t y = 0; y < ny; ++y)
      for (int64_t x = 0; x < nx; ++x) {
        const int64_t n = x + nx * (y + ny * z);
        if (!(phi[n] < thr)) continue;  /* not a bulk node */
        for (int a = 0; a < L->q; ++a) {
          const int b = L->opp[a];
          if (b <= a) continue;  /* each pair of opposite directions once; skips rest */
          int64_t ip, im;
          if (!sample_point(p, x, y, z, L->c[a], d, &ip)) continue;
          if (!sample_point(p, x, y, z, L->c[b], d, &im)) continue;
          if (phi[ip] > thr && phi[im] > thr) {
            flag[ip] = 1;
            flag[im] = 1;
          }
        }
      }
}

/* ------------------------------------------------------------------------ */
/* Exported API                                                              */
/* ------------------------------------------------------------------------ */

int ref_lattice(int kind, int* q, int* d, int* c, double* w, int* opp) {
  lattice_t L;
  if (build_lattice(kind, &L) != 0) return -1;
  *q = L.q;
  *d = L.d;
  for (int a = 0; a < L.q; ++a) {
    for (int al = 0; al < 3; ++al) c[a * 3 + al] = L.c[a][al];
    w[a] = L.w[a];
    opp[a] = L.opp[a];
  }
  return 0;
}

int ref_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* f = f^eq(rho, u) for every node (species 1), or the colour split
 * f_R = (rho_R/rho) f^eq, f_B = (rho_B/rho) f^eq with
 * rho_R = rho (1 + phi)/2, rho_B = rho (1 - phi)/2 (species 2).
 * rho[N], u[D*N] SoA, phi[N] (species 2 only).  f[species*Q*N]. */
int ref_init(const ref_params* p, const double* rho, const double* u, const double* phi,
             double* f) {
  lattice_t L;
  if (check_params(p, &L) != 0) return -1;
  const int64_t N = p->nx * p->ny * p->nz;
  const int Q = L.q, D = L.d;
#pragma omp parallel for schedule(static) if (N >= OMP_MIN_NODES)
  for (int64_t n = 0; n < N; ++n) {
    double uu[3] = {0.0, 0.0, 0.0};
    for (int al = 0; al < D; ++al) uu[al] = u[(int64_t)al * N + n];
    double feq[27];
    equilibrium(&L, p, rho[n], uu, feq);
    if (p->species == 1) {
      for (int a = 0; a < Q; ++a) f[(int64_t)a * N + n] = feq[a];
    } else {
      double xr = 0.5 * (1.0 + phi[n]), xb = 0.5 * (1.0 - phi[n]);
      for (int a = 0; a < Q; ++a) {
        f[(int64_t)a * N + n] = xr * feq[a];
        f[(int64_t)(Q + a) * N + n] = xb * feq[a];
      }
    }
  }
  return 0;
}

/* One regularized step, single species: f -> fnew (two arrays, push). */
static void step_one_species(const lattice_t* L, const ref_params* p, const double* f,
                             double* fnew) {
  const int64_t nx = p->nx, ny = p->ny, nz = p->nz;
  const int64_t N = nx * ny * nz;
  const int Q = L->q;
#pragma omp parallel for collapse(2) schedule(static) if (N >= OMP_MIN_NODES)
  for (int64_t z = 0; z < nz; ++z)
    for (int64_t y = 0; y < ny; ++y)
      for (int64_t x = 0; x < nx; ++x) {
        const int64_t n = x + nx * (y + ny * z);
        double fl[27], fpc[27];
        for (int a = 0; a < Q; ++a) fl[a] = f[(int64_t)a * N + n];
        collide(L, p, fl, fpc);
        for (int a = 0; a < Q; ++a) {
          int64_t t;
          if (destination(L, p, a, x, y, z, &t))
            fnew[(int64_t)a * N + t] = fpc[a];
          else
            fnew[(int64_t)L->opp[a] * N + n] = fpc[a] + wall_term(L, p, a, x, y, z);
        }
      }
}

/* One colour-gradient step, two species: f[2][Q][N] -> fnew.  flag[N] is
 * scratch for the near-contact flags (NULL when they are off). */
static void step_two_species(const lattice_t* L, const ref_params* p, const double* f,
                             double* fnew, double* phi, unsigned char* flag) {
  const int64_t nx = p->nx, ny = p->ny, nz = p->nz;
  const int64_t N = nx * ny * nz;
  const int Q = L->q;
  const double omega = 1.0 / p->tau;
  double B[27];
  weights_B(L, B);
  phase_field(L, p, f, N, phi);
  if (flag) nci_flags(L, p, phi, flag);
#pragma omp parallel for collapse(2) schedule(static) if (N >= OMP_MIN_NODES)
  for (int64_t z = 0; z < nz; ++z)
    for (int64_t y = 0; y < ny; ++y)
      for (int64_t x = 0; x < nx; ++x) {
        const int64_t n = x + nx * (y + ny * z);
        double g[27], gpc[27], rr = 0.0, rb = 0.0;
        for (int a = 0; a < Q; ++a) {
          double fr = f[(int64_t)a * N + n], fb = f[(int64_t)(Q + a) * N + n];
          g[a] = fr + fb;
          rr += fr;
          rb += fb;
        }
        const double rho = rr + rb;
        double G[3];
        gradient(L, p, phi, x, y, z, G);
        const double G2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
        const double Gn = sqrt(G2);
        double Ft[3] = {p->force[0], p->force[1], p->force[2]};
        if (flag && flag[n] && G2 > 1e-20)
          for (int al = 0; al < 3; ++al) Ft[al] += p->nci_strength * rr * G[al] / Gn;
        collide_f(L, p, g, Ft, gpc);
        for (int a = 0; a < Q; ++a) {
          double cG = cdot(L, a, G);
          double c2 = (double)(L->c[a][0] * L->c[a][0] + L->c[a][1] * L->c[a][1] +
                               L->c[a][2] * L->c[a][2]);
          double pert = 0.0, cosang = 0.0;
          if (G2 > 1e-20) {
            pert = 2.25 * p->sigma * omega * Gn * (L->w[a] * cG * cG / G2 - B[a]);
            if (c2 > 0.0) cosang = cG / (sqrt(c2) * Gn);
          }
          const double gs = gpc[a] + pert;
          const double rec = p->beta * (rr * rb / rho) * L->w[a] * cosang;
          const double out[2] = {(rr / rho) * gs + rec, (rb / rho) * gs - rec};
          int64_t t;
          int inside = destination(L, p, a, x, y, z, &t);
          for (int s = 0; s < 2; ++s) {
            if (inside)
              fnew[(int64_t)(s * Q + a) * N + t] = out[s];
            else
              fnew[(int64_t)(s * Q + L->opp[a]) * N + n] = out[s];
          }
        }
      }
}

/* Advance f in place by nsteps steps.  f has species*Q*N doubles. */
int ref_run(const ref_params* p, double* f, int64_t nsteps) {
  lattice_t L;
  if (check_params(p, &L) != 0) return -1;
  const int64_t N = p->nx * p->ny * p->nz;
  const int64_t total = (int64_t)p->species * L.q * N;
  double* fb = (double*)malloc((size_t)total * sizeof(double));
  double* phi = (p->species == 2) ? (double*)malloc((size_t)N * sizeof(double)) : NULL;
  const int nci = p->species == 2 && p->nci_strength != 0.0;
  unsigned char* flag = nci ? (unsigned char*)malloc((size_t)N) : NULL;
  if (!fb || (p->species == 2 && !phi) || (nci && !flag)) {
    free(fb);
    free(phi);
    free(flag);
    return -2;
  }
  double* cur = f;
  double* nxt = fb;
  for (int64_t s = 0; s < nsteps; ++s) {
    if (p->species == 1)
      step_one_species(&L, p, cur, nxt);
    else
      step_two_species(&L, p, cur, nxt, phi, flag);
    double* t = cur;
    cur = nxt;
    nxt = t;
  }
  if (cur != f) memcpy(f, cur, (size_t)total * sizeof(double));
  free(fb);
  free(phi);
  free(flag);
  return 0;
}

/* Near-contact flags and forces of the current two-species populations f:
 * flag[N] (0/1) from the flagging pass, force[3 N] (x, then y, then z) the
 * near-contact force of each node (without the constant body force). */
int ref_nci(const ref_params* p, const double* f, unsigned char* flag, double* force) {
  lattice_t L;
  if (check_params(p, &L) != 0 || p->species != 2) return -1;
  const int64_t nx = p->nx, ny = p->ny, nz = p->nz;
  const int64_t N = nx * ny * nz;
  const int Q = L.q;
  double* phi = (double*)malloc((size_t)N * sizeof(double));
  if (!phi) return -2;
  phase_field(&L, p, f, N, phi);
  nci_flags(&L, p, phi, flag);
  for (int64_t z = 0; z < nz; ++z)
    for (int64_t y = 0; y < ny; ++y)
      for (int64_t x = 0; x < nx; ++x) {
        const int64_t n = x + nx * (y + ny * z);
        double G[3], rr = 0.0;
        for (int a = 0; a < Q; ++a) rr += f[(int64_t)a * N + n];
        gradient(&L, p, phi, x, y, z, G);
        const double G2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
        for (int al = 0; al < 3; ++al) {
          force[(int64_t)al * N + n] = 0.0;
          if (flag[n] && G2 > 1e-20)
            force[(int64_t)al * N + n] = p->nci_strength * rr * G[al] / sqrt(G2);
        }
      }
  free(phi);
  return 0;
}

/* Moments of the current populations: rho[N], u[D*N] = (j + F/2)/rho0,
 * pineq[D(D+1)/2 * N] = sum_a (f_a - f^eq_a) c_a c_a ordered xx,yy,(zz),xy,(xz,yz),
 * phi[N] for two species (may be NULL).  For two species the moments are
 * those of g = f_R + f_B. */
int ref_moments(const ref_params* p, const double* f, double* rho, double* u, double* pineq,
                double* phi) {
  lattice_t L;
  if (check_params(p, &L) != 0) return -1;
  const int64_t N = p->nx * p->ny * p->nz;
  const int Q = L.q, D = L.d;
#pragma omp parallel for schedule(static) if (N >= OMP_MIN_NODES)
  for (int64_t n = 0; n < N; ++n) {
    double fl[27], rr = 0.0, rb = 0.0;
    for (int a = 0; a < Q; ++a) {
      fl[a] = f[(int64_t)a * N + n];
      rr += fl[a];
      if (p->species == 2) {
        double fbv = f[(int64_t)(Q + a) * N + n];
        fl[a] += fbv;
        rb += fbv;
      }
    }
    double r, j[3], uu[3], feq[27];
    node_moments(&L, p, fl, &r, j, uu);
    equilibrium(&L, p, r, uu, feq);
    double Pi[3][3] = {{0.0}};
    for (int a = 0; a < Q; ++a)
      for (int al = 0; al < 3; ++al)
        for (int be = 0; be < 3; ++be) Pi[al][be] += (fl[a] - feq[a]) * L.c[a][al] * L.c[a][be];
    if (rho) rho[n] = r;
    if (u)
      for (int al = 0; al < D; ++al) u[(int64_t)al * N + n] = uu[al];
    if (pineq) {
      if (D == 2) {
        pineq[n] = Pi[0][0];
        pineq[N + n] = Pi[1][1];
        pineq[2 * N + n] = Pi[0][1];
      } else {
        pineq[n] = Pi[0][0];
        pineq[N + n] = Pi[1][1];
        pineq[2 * N + n] = Pi[2][2];
        pineq[3 * N + n] = Pi[0][1];
        pineq[4 * N + n] = Pi[0][2];
        pineq[5 * N + n] = Pi[1][2];
      }
    }
    if (phi && p->species == 2) phi[n] = (rr - rb) / (rr + rb);
  }
  return 0;
}

/* Single-node regularized collision (single species), for identity tests. */
int ref_collide_node(const ref_params* p, const double* f, double* fpc) {
  lattice_t L;
  if (build_lattice(p->lattice, &L) != 0) return -1;
  collide(&L, p, f, fpc);
  return 0;
}

/* Single-node equilibrium, for identity tests. */
int ref_equilibrium_node(const ref_params* p, double rho, const double* u, double* feq) {
  lattice_t L;
  if (build_lattice(p->lattice, &L) != 0) return -1;
  double uu[3] = {u[0], u[1], L.d == 3 ? u[2] : 0.0};
  equilibrium(&L, p, rho, uu, feq);
  return 0;
}
