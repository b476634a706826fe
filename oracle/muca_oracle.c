/*
 * FP64 reference oracle for multicanonical (MUCA) Metropolis sampling of coarse-grained
 * AB heteropolymers -- TEST INFRASTRUCTURE ONLY.
 *
 * Written from Frigori, "PHAST: Protein-like Heteropolymer Analysis by Statistical
 * Thermodynamics" (arXiv:1702.01770).  Plain, serial, double precision, no blocking and no
 * reordering beyond what each definition states, so that every function can be read against
 * the paper:
 *   - couplings C_LJ(sigma_i, sigma_j)                         Eq. (1)
 *   - single-chain energy (bending + intra-chain LJ)            Eq. (2), AB limit kappa_F = 0
 *   - multi-chain energy (inter-chain LJ)                      Eq. (3)
 *   - MUCA weights ln W(E) = -beta_k E + alpha_k               Eq. (8)
 *   - Metropolis with MUCA weights, histogram at every step     Sec. 2.2 and Sec. 3.2
 *   - iterative weight estimate, Berg's accumulated recursion  Sec. 2.2
 * Readings where the paper is silent (torsion term, move set, window, bins, RNG) are the ones
 * listed in the design notes of this repository; each is restated at the function using it.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may load this
 * library.  It shares no code with the HIP library.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",  */
/* SC'11).  Counter-based: out = f_key(counter).  The paper's package draws uniforms from     */
/* cuRAND vectors (Sec. 3.2, RANDOM.f / cudaRandom.cu); this implementation draws one Philox   */
/* block per trial move instead, so that CPU and GPU can draw identical streams.              */
/* ------------------------------------------------------------------------------------------ */
static const uint32_t PHILOX_M0 = 0xD2511F53u, PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u, PHILOX_W1 = 0xBB67AE85u;

void orc_philox(uint32_t k0, uint32_t k1, const uint32_t ctr_in[4], uint32_t out[4])
{
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
        uint64_t p0 = (uint64_t)PHILOX_M0 * c[0];
        uint64_t p1 = (uint64_t)PHILOX_M1 * c[2];
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    }
    memcpy(out, c, sizeof c);
}

void orc_philox_many(int64_t n, const uint32_t *k0, const uint32_t *k1, const uint32_t *ctr,
                     uint32_t *out)
{
    for (int64_t i = 0; i < n; ++i) orc_philox(k0[i], k1[i], ctr + 4 * i, out + 4 * i);
}

/* Uniform in (0,1) from a 32-bit word: (x + 1/2) 2^-32, exact in FP64. */
static double u01(uint32_t x) { return ((double)x + 0.5) * (1.0 / 4294967296.0); }

/* Stream key of a walker: (low word of the seed, high word of the seed XOR walker id). */
static void walker_key(uint64_t seed, uint32_t walker, uint32_t *k0, uint32_t *k1)
{
    *k0 = (uint32_t)seed;
    *k1 = (uint32_t)(seed >> 32) ^ walker;
}

/* ------------------------------------------------------------------------------------------ */
/* System description and energy                                                              */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    int32_t n_beads, n_chains, n_types, box_kind;  /* 0 none, 1 steric sphere, 2 periodic cube */
    const int32_t *chain_start;                     /* n_chains + 1 bead offsets */
    const uint8_t *type;                            /* n_beads letters, < n_types */
    const double *c_lj;                             /* n_types x n_types, Eq. (1) */
    double k_intra, k_inter, k_bend, k_tors;
    double box_len;                                 /* cube edge, or sphere radius */
} orc_system;

/* Steric sphere of radius box_len about the origin (the container of the paper's simulations,
 * Sec. 4): a bead may not leave it, so a trial move that would take one outside is rejected. */
static int outside_sphere(const orc_system *s, const double *x)
{
    if (s->box_kind != 1) return 0;
    return x[0] * x[0] + x[1] * x[1] + x[2] * x[2] > s->box_len * s->box_len;
}

typedef struct {
    double e_lo, bin_width;
    int32_t n_bins;
    const double *beta, *alpha;  /* ln W(E) = -beta[k] E + alpha[k], k = bin of E (Eq. 8) */
    double edge_tol;             /* a starting energy up to edge_tol outside the window is
                                    counted in the edge bin (0: none); see start_bin */
} orc_weights;

typedef struct {
    double crank_max;        /* interior bead: rotation angle uniform in [-crank_max, crank_max] */
    double cap_rho;          /* end bead: new bond along d + rho g, g uniform on the unit sphere */
    double trans_max;        /* rigid chain translation: each axis uniform in [-t, t] */
    int32_t rigid_per_sweep; /* rigid translations after every sweep (multi-chain systems) */
    int32_t pivot_per_sweep; /* pivots after every sweep */
    double pivot_max;        /* pivot angle uniform in [-pivot_max, pivot_max] */
    int32_t rotate_per_sweep;/* rigid chain rotations about the chain centre (multi-chain) */
    double rotate_max;       /* rotation angle uniform in [-rotate_max, rotate_max] */
} orc_moves;

static int chain_of(const orc_system *s, int b)
{
    int c = 0;
    while (s->chain_start[c + 1] <= b) ++c;
    return c;
}

/* Separation vector x_i - x_j; in the periodic cube each axis takes its minimum image. */
static void separation(const orc_system *s, const double *xi, const double *xj, double d[3])
{
    for (int a = 0; a < 3; ++a) {
        double v = xi[a] - xj[a];
        if (s->box_kind == 2) v -= s->box_len * rint(v / s->box_len);
        d[a] = v;
    }
}

/* Non-bonded pair term of Eqs. (2)-(3): kappa (r^-12 - C r^-6).  *scale gets the magnitude
 * kappa (r^-12 + |C| r^-6) used as the size of the term in error bounds. */
static double pair_term(const orc_system *s, int i, int j, const double *xi, const double *xj,
                        int same_chain, double *scale)
{
    double d[3];
    separation(s, xi, xj, d);
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double inv6 = 1.0 / (r2 * r2 * r2);
    double c = s->c_lj[s->type[i] * s->n_types + s->type[j]];
    double kappa = same_chain ? s->k_intra : s->k_inter;
    if (scale) *scale = kappa * (inv6 * inv6 + fabs(c) * inv6);
    return kappa * (inv6 * inv6 - c * inv6);
}

static void unit_bond(const double *from, const double *to, double u[3])
{
    double b[3] = {to[0] - from[0], to[1] - from[1], to[2] - from[2]};
    double n = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    u[0] = b[0] / n; u[1] = b[1] / n; u[2] = b[2] / n;
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Bending term at the angle between bonds (i, i+1) and (i+1, i+2) of one chain: Eq. (2),
 * kappa_C (1 - cos theta) with cos theta the cosine between the normalised bond vectors. */
static double bend_term(const orc_system *s, const double *pos, int i)
{
    double u1[3], u2[3];
    unit_bond(pos + 3 * i, pos + 3 * (i + 1), u1);
    unit_bond(pos + 3 * (i + 1), pos + 3 * (i + 2), u2);
    return s->k_bend * (1.0 - dot3(u1, u2));
}

/* Torsion-like term between bonds (i, i+1) and (i+2, i+3): kappa_T (1 - u_i . u_{i+2}).  Not in
 * the paper's Eq. (2) (kappa_T = 0 recovers it); it is the next-nearest-bond coupling of the 3D
 * off-lattice AB model. */
static double tors_term(const orc_system *s, const double *pos, int i)
{
    double u1[3], u3[3];
    unit_bond(pos + 3 * i, pos + 3 * (i + 1), u1);
    unit_bond(pos + 3 * (i + 2), pos + 3 * (i + 3), u3);
    return s->k_tors * (1.0 - dot3(u1, u3));
}

/* Full energy E(x) = sum over chains of H_single (Eq. 2) + inter-chain LJ (Eq. 3).
 * parts[0..3] (optional) = bending, torsion, intra LJ, inter LJ; *abs_scale (optional) = sum of
 * the magnitudes of all individual terms. */
double orc_energy(const orc_system *s, const double *pos, double parts[4], double *abs_scale)
{
    double bend = 0, tors = 0, intra = 0, inter = 0, scale = 0;
    for (int c = 0; c < s->n_chains; ++c) {
        int first = s->chain_start[c], last = s->chain_start[c + 1] - 1;
        for (int i = first; i + 2 <= last; ++i) { double t = bend_term(s, pos, i); bend += t; scale += fabs(t); }
        for (int i = first; i + 3 <= last; ++i) { double t = tors_term(s, pos, i); tors += t; scale += fabs(t); }
    }
    for (int i = 0; i < s->n_beads; ++i) {
        int ci = chain_of(s, i);
        for (int j = i + 1; j < s->n_beads; ++j) {
            int cj = chain_of(s, j);
            if (ci == cj && j == i + 1) continue;          /* bonded neighbours: no LJ term */
            double sc;
            double t = pair_term(s, i, j, pos + 3 * i, pos + 3 * j, ci == cj, &sc);
            if (ci == cj) intra += t; else inter += t;
            scale += sc;
        }
    }
    if (parts) { parts[0] = bend; parts[1] = tors; parts[2] = intra; parts[3] = inter; }
    if (abs_scale) *abs_scale = scale;
    return bend + tors + intra + inter;
}

/* Sum of every energy term that contains bead b (pairs with b, bends and torsions whose bonds
 * end at b).  E(x') - E(x) for a move of bead b equals the difference of this quantity. */
static double terms_with_bead(const orc_system *s, const double *pos, int b)
{
    int c = chain_of(s, b);
    int first = s->chain_start[c], last = s->chain_start[c + 1] - 1;
    double e = 0;
    for (int j = 0; j < s->n_beads; ++j) {
        if (j == b) continue;
        int cj = chain_of(s, j);
        if (cj == c && (j == b - 1 || j == b + 1)) continue;
        e += pair_term(s, b, j, pos + 3 * b, pos + 3 * j, cj == c, NULL);
    }
    for (int i = b - 2; i <= b; ++i)               /* bends using bond b-1 or bond b */
        if (i >= first && i + 2 <= last) e += bend_term(s, pos, i);
    for (int i = b - 3; i <= b; ++i)               /* torsions using bond b-1 or bond b */
        if (i >= first && i + 3 <= last && (i == b - 1 || i == b || i + 2 == b - 1 || i + 2 == b))
            e += tors_term(s, pos, i);
    return e;
}

/* Inter-chain LJ energy between chain c and all other chains (Eq. 3), the only part of E that a
 * rigid translation of chain c changes. */
static double inter_terms_of_chain(const orc_system *s, const double *pos, int c)
{
    double e = 0;
    for (int i = s->chain_start[c]; i < s->chain_start[c + 1]; ++i)
        for (int j = 0; j < s->n_beads; ++j) {
            if (j >= s->chain_start[c] && j < s->chain_start[c + 1]) continue;
            e += pair_term(s, i, j, pos + 3 * i, pos + 3 * j, 0, NULL);
        }
    return e;
}

/* ------------------------------------------------------------------------------------------ */
/* Trial moves (paper: spherical caps, pivots, Galilean updates, Sec. 3.2).  This code moves   */
/* one bead at a time and keeps every bond at r0 = 1 (AB limit, kappa_F = 0), so Delta E is    */
/* O(N).  Both proposals are symmetric, hence plain Metropolis acceptance is exact.            */
/* ------------------------------------------------------------------------------------------ */

/* End bead b with bonded neighbour a: d = x_b - x_a (unit), g uniform on the unit sphere from
 * (u1, u2); the new bead sits at x_a + (d + rho g)/|d + rho g|. */
static void propose_end(const double *xa, const double *xb, double rho, double u1, double u2,
                        double out[3])
{
    double z = 2.0 * u1 - 1.0;
    double psi = 2.0 * M_PI * u2;
    double sxy = sqrt(fmax(0.0, 1.0 - z * z));
    double g[3] = {sxy * cos(psi), sxy * sin(psi), z};
    double v[3];
    for (int a = 0; a < 3; ++a) v[a] = (xb[a] - xa[a]) + rho * g[a];
    double n = sqrt(dot3(v, v));
    for (int a = 0; a < 3; ++a) out[a] = xa[a] + v[a] / n;
}

/* Interior bead b: crankshaft rotation of x_b about the axis through x_{b-1} and x_{b+1} by
 * phi = crank_max (2 u1 - 1) (Rodrigues' formula).  Both bond lengths are preserved. */
static void propose_crank(const double *xp, const double *xb, const double *xn, double phi,
                          double out[3])
{
    double a[3] = {xn[0] - xp[0], xn[1] - xp[1], xn[2] - xp[2]};
    double na = sqrt(dot3(a, a));
    double k[3] = {a[0] / na, a[1] / na, a[2] / na};
    double v[3] = {xb[0] - xp[0], xb[1] - xp[1], xb[2] - xp[2]};
    double c = cos(phi), sn = sin(phi);
    double kxv[3] = {k[1] * v[2] - k[2] * v[1], k[2] * v[0] - k[0] * v[2], k[0] * v[1] - k[1] * v[0]};
    double kv = dot3(k, v);
    for (int i = 0; i < 3; ++i) out[i] = xp[i] + (v[i] * c + kxv[i] * sn + k[i] * kv * (1.0 - c));
}

/* Bin of energy E in the window [e_lo, e_lo + n_bins * bin_width); -1 outside.  The bin is
 * floor((E - e_lo) * (1 / bin_width)) with the reciprocal rounded once: at a bin edge a quotient
 * and this product may differ by one bin, and both implementations quantise this way. */
static int64_t bin_of(const orc_weights *w, double e)
{
    double t = (e - w->e_lo) * (1.0 / w->bin_width);
    if (!(t >= 0.0) || !(t < (double)w->n_bins)) return -1;
    return (int64_t)floor(t);
}

/* Bin of a walker's starting energy: its bin inside the window; otherwise, when the energy lies at
 * most edge_tol outside it, the edge bin on that side (ln W then extends that bin's line); -1
 * beyond.  This is the window-edge reading for energies that reduced-precision accumulation can
 * leave just outside the window; with edge_tol = 0 it is bin_of. */
static int64_t start_bin(const orc_weights *w, double e)
{
    int64_t k = bin_of(w, e);
    if (k >= 0 || !(w->edge_tol > 0.0)) return k;
    const double top = w->e_lo + (double)w->n_bins * w->bin_width;
    if (e >= w->e_lo - w->edge_tol && e < top + w->edge_tol)
        return (e - w->e_lo) * (1.0 / w->bin_width) < 0.0 ? 0 : w->n_bins - 1;
    return -1;
}

/* ln W(E) of Eq. (8), continuous and piecewise linear in E. */
static double ln_weight(const orc_weights *w, double e, int64_t k)
{
    return -w->beta[k] * e + w->alpha[k];
}

/* Metropolis test with MUCA weights: accept iff E' lies in the window and
 * ln u < ln W(E') - ln W(E), i.e. u < W(E')/W(E). */
static int metropolis(const orc_weights *w, double e_old, int64_t k_old, double e_new, double u,
                      int64_t *k_new)
{
    int64_t k = bin_of(w, e_new);
    *k_new = k;
    if (k < 0) return 0;
    double delta = ln_weight(w, e_new, k) - ln_weight(w, e_old, k_old);
    return log(u) < delta;
}

typedef struct {
    int64_t moves, accepted;             /* single-bead trial moves */
    int64_t rigid_moves, rigid_accepted; /* rigid chain translations */
    int64_t window_rejects;              /* proposals rejected for leaving the window */
    double max_drift;                    /* max |E_running - E_full| seen at checks */
    int64_t pivot_moves, pivot_accepted; /* pivots */
    int64_t rot_moves, rot_accepted;     /* rigid chain rotations */
} orc_counters;

/* Unit vector from two uniforms: z = 2 u1 - 1, azimuth 2 pi u2 (uniform on the sphere). */
static void unit_from(double u1, double u2, double k[3])
{
    double z = 2.0 * u1 - 1.0;
    double psi = 2.0 * M_PI * u2;
    double sxy = sqrt(fmax(0.0, 1.0 - z * z));
    k[0] = sxy * cos(psi); k[1] = sxy * sin(psi); k[2] = z;
}

/* x -> c + R (x - c): rotation by phi about the unit axis k through the point c (Rodrigues). */
static void rotate_about(const double c[3], const double k[3], double phi, double *x)
{
    double v[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
    double co = cos(phi), sn = sin(phi);
    double kxv[3] = {k[1] * v[2] - k[2] * v[1], k[2] * v[0] - k[0] * v[2], k[0] * v[1] - k[1] * v[0]};
    double kv = dot3(k, v);
    for (int i = 0; i < 3; ++i) x[i] = c[i] + (v[i] * co + kxv[i] * sn + k[i] * kv * (1.0 - co));
}

/* Chain-level trial move on beads [lo, hi]: rotate them by phi about the axis k through c,
 * accept with the Metropolis-MUCA test using Delta E = E(x') - E(x) (full energies), restore
 * them if rejected.  Returns 1 if accepted; *k_new as for metropolis. */
static int rotate_block(const orc_system *s, const orc_weights *w, double *pos, int lo, int hi,
                        const double c[3], const double k[3], double phi, double u, double *e,
                        int64_t *kb, int64_t *k_new)
{
    int nb = hi - lo + 1;
    double *keep = (double *)malloc(sizeof(double) * 3 * (size_t)nb);
    memcpy(keep, pos + 3 * lo, sizeof(double) * 3 * (size_t)nb);
    double before = orc_energy(s, pos, NULL, NULL);
    for (int i = lo; i <= hi; ++i) rotate_about(c, k, phi, pos + 3 * i);
    double after = orc_energy(s, pos, NULL, NULL);
    double e_new = *e + (after - before);
    int acc = metropolis(w, *e, *kb, e_new, u, k_new);
    for (int i = lo; i <= hi; ++i)
        if (outside_sphere(s, pos + 3 * i)) acc = 0;
    if (acc) { *e = e_new; *kb = *k_new; }
    else memcpy(pos + 3 * lo, keep, sizeof(double) * 3 * (size_t)nb);
    free(keep);
    return acc;
}

/*
 * Run one walker for n_sweeps sweeps (Sec. 2.2 / 3.2, MONTE_CARLO).  A sweep is N single-bead
 * trial moves; move m of the walker's sweep number S uses the Philox block at counter
 * (m, lo32(S), hi32(S), 0) under the walker's key: word 0 picks the bead (x0 * N) >> 32, words
 * 1-2 drive the proposal and word 3 the acceptance.  After the N moves of a multi-chain system
 * come rigid_per_sweep chain translations drawn from counters (r, lo, hi, 1) (chain and shift)
 * and (r, lo, hi, 2) (acceptance).  Then pivot_per_sweep pivots (the paper's pivotings): the
 * block at (r, lo, hi, 3) picks the pivot bead p = (x0 * N) >> 32, the axis (words 1-2, uniform
 * on the sphere) and the angle (word 3, uniform in +-pivot_max); the block at (r, lo, hi, 4)
 * gives the acceptance (word 0) and the side (word 1 < 2^31: the beads after p in its chain,
 * else those before it; for a chain end, the side that has beads), which is rotated about x_p.
 * Then, for multi-chain systems, rotate_per_sweep rigid rotations of a chain (the paper's
 * Galilean rotations) about its centre: blocks (r, lo, hi, 5) (chain (x0 * M) >> 32, axis,
 * angle in +-rotate_max) and (r, lo, hi, 6) (acceptance).  After every trial move, accepted or
 * not, the bin of the current energy is counted in hist (the paper updates the histogram at
 * every simulation step).
 *
 * pos (N x 3) and *energy are updated in place; *sweep_counter advances by n_sweeps.
 * accept_log (optional, capacity log_cap bytes) gets one byte per single-bead trial move
 * (1 accepted, 0 rejected).  check_every > 0 recomputes the full energy every check_every
 * trial moves and records the largest |E_running - E_full| in counters->max_drift.
 * Returns 0, or -1 if the starting energy lies outside the window.
 */
int orc_run(const orc_system *s, const orc_weights *w, const orc_moves *mv, uint64_t seed,
            uint32_t walker, uint64_t *sweep_counter, double *pos, double *energy,
            int64_t n_sweeps, uint64_t *hist, uint8_t *accept_log, int64_t log_cap,
            int64_t check_every, orc_counters *cnt)
{
    uint32_t k0, k1;
    walker_key(seed, walker, &k0, &k1);
    const int n = s->n_beads;
    double e = *energy;
    int64_t k = start_bin(w, e);
    if (k < 0) return -1;
    double newpos[3], saved[3];
    int64_t logged = 0, since_check = 0;

    for (int64_t sw = 0; sw < n_sweeps; ++sw) {
        uint64_t S = *sweep_counter;
        for (int m = 0; m < n; ++m) {
            uint32_t ctr[4] = {(uint32_t)m, (uint32_t)S, (uint32_t)(S >> 32), 0u}, r[4];
            orc_philox(k0, k1, ctr, r);
            int b = (int)(((uint64_t)r[0] * (uint64_t)n) >> 32);
            int c = chain_of(s, b);
            int first = s->chain_start[c], last = s->chain_start[c + 1] - 1;
            double *xb = pos + 3 * b;
            if (b == first || b == last) {
                int a = (b == first) ? b + 1 : b - 1;
                propose_end(pos + 3 * a, xb, mv->cap_rho, u01(r[1]), u01(r[2]), newpos);
            } else {
                double phi = mv->crank_max * (2.0 * u01(r[1]) - 1.0);
                propose_crank(pos + 3 * (b - 1), xb, pos + 3 * (b + 1), phi, newpos);
            }
            double before = terms_with_bead(s, pos, b);
            memcpy(saved, xb, sizeof saved);
            memcpy(xb, newpos, sizeof newpos);
            double after = terms_with_bead(s, pos, b);
            double e_new = e + (after - before);
            int64_t k_new;
            int acc = metropolis(w, e, k, e_new, u01(r[3]), &k_new);
            if (outside_sphere(s, newpos)) acc = 0;
            if (acc) { e = e_new; k = k_new; cnt->accepted++; }
            else {
                memcpy(xb, saved, sizeof saved);
                if (k_new < 0) cnt->window_rejects++;
            }
            cnt->moves++;
            hist[k] += 1;
            if (accept_log && logged < log_cap) accept_log[logged++] = (uint8_t)acc;
            if (check_every > 0 && ++since_check == check_every) {
                since_check = 0;
                double d = fabs(e - orc_energy(s, pos, NULL, NULL));
                if (d > cnt->max_drift) cnt->max_drift = d;
            }
        }
        if (s->n_chains > 1) {
            for (int rr = 0; rr < mv->rigid_per_sweep; ++rr) {
                uint32_t c1[4] = {(uint32_t)rr, (uint32_t)S, (uint32_t)(S >> 32), 1u}, r1[4];
                uint32_t c2[4] = {(uint32_t)rr, (uint32_t)S, (uint32_t)(S >> 32), 2u}, r2[4];
                orc_philox(k0, k1, c1, r1);
                orc_philox(k0, k1, c2, r2);
                int ch = (int)(((uint64_t)r1[0] * (uint64_t)s->n_chains) >> 32);
                double delta[3];
                for (int a = 0; a < 3; ++a) delta[a] = mv->trans_max * (2.0 * u01(r1[1 + a]) - 1.0);
                double before = inter_terms_of_chain(s, pos, ch);
                int c0 = s->chain_start[ch], nc = s->chain_start[ch + 1] - c0;
                double *keep = (double *)malloc(sizeof(double) * 3 * (size_t)nc);
                memcpy(keep, pos + 3 * c0, sizeof(double) * 3 * (size_t)nc);
                for (int i = s->chain_start[ch]; i < s->chain_start[ch + 1]; ++i)
                    for (int a = 0; a < 3; ++a) pos[3 * i + a] += delta[a];
                double after = inter_terms_of_chain(s, pos, ch);
                double e_new = e + (after - before);
                int64_t k_new;
                int acc = metropolis(w, e, k, e_new, u01(r2[0]), &k_new);
                for (int i = s->chain_start[ch]; i < s->chain_start[ch + 1]; ++i)
                    if (outside_sphere(s, pos + 3 * i)) acc = 0;
                if (acc) { e = e_new; k = k_new; cnt->rigid_accepted++; }
                else {
                    memcpy(pos + 3 * c0, keep, sizeof(double) * 3 * (size_t)nc);
                    if (k_new < 0) cnt->window_rejects++;
                }
                free(keep);
                cnt->rigid_moves++;
                hist[k] += 1;
            }
        }
        for (int rr = 0; rr < mv->pivot_per_sweep; ++rr) {
            uint32_t ca[4] = {(uint32_t)rr, (uint32_t)S, (uint32_t)(S >> 32), 3u}, ra[4];
            uint32_t cb[4] = {(uint32_t)rr, (uint32_t)S, (uint32_t)(S >> 32), 4u}, rb[4];
            orc_philox(k0, k1, ca, ra);
            orc_philox(k0, k1, cb, rb);
            int p = (int)(((uint64_t)ra[0] * (uint64_t)n) >> 32);
            int c = chain_of(s, p);
            int first = s->chain_start[c], last = s->chain_start[c + 1] - 1;
            int tail = (p == first) ? 1 : (p == last) ? 0 : (rb[1] < 0x80000000u);
            int lo = tail ? p + 1 : first, hi = tail ? last : p - 1;
            double axis[3], ctr[3] = {pos[3 * p], pos[3 * p + 1], pos[3 * p + 2]};
            unit_from(u01(ra[1]), u01(ra[2]), axis);
            double phi = mv->pivot_max * (2.0 * u01(ra[3]) - 1.0);
            int64_t k_new;
            int acc = rotate_block(s, w, pos, lo, hi, ctr, axis, phi, u01(rb[0]), &e, &k, &k_new);
            if (acc) cnt->pivot_accepted++;
            else if (k_new < 0) cnt->window_rejects++;
            cnt->pivot_moves++;
            hist[k] += 1;
        }
        if (s->n_chains > 1) {
            for (int rr = 0; rr < mv->rotate_per_sweep; ++rr) {
                uint32_t ca[4] = {(uint32_t)rr, (uint32_t)S, (uint32_t)(S >> 32), 5u}, ra[4];
                uint32_t cb[4] = {(uint32_t)rr, (uint32_t)S, (uint32_t)(S >> 32), 6u}, rb[4];
                orc_philox(k0, k1, ca, ra);
                orc_philox(k0, k1, cb, rb);
                int ch = (int)(((uint64_t)ra[0] * (uint64_t)s->n_chains) >> 32);
                int lo = s->chain_start[ch], hi = s->chain_start[ch + 1] - 1;
                double ctr[3] = {0, 0, 0}, axis[3];
                for (int i = lo; i <= hi; ++i)
                    for (int a = 0; a < 3; ++a) ctr[a] += pos[3 * i + a];
                for (int a = 0; a < 3; ++a) ctr[a] /= (double)(hi - lo + 1);
                unit_from(u01(ra[1]), u01(ra[2]), axis);
                double phi = mv->rotate_max * (2.0 * u01(ra[3]) - 1.0);
                int64_t k_new;
                int acc = rotate_block(s, w, pos, lo, hi, ctr, axis, phi, u01(rb[0]), &e, &k, &k_new);
                if (acc) cnt->rot_accepted++;
                else if (k_new < 0) cnt->window_rejects++;
                cnt->rot_moves++;
                hist[k] += 1;
            }
        }
        *sweep_counter = S + 1;
    }
    *energy = e;
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Weight recursion between iterations (Sec. 2.2): start from W = 1 (beta = alpha = 0), the     */
/* first iteration is the simple recursion W^{n+1} = W^n / H^n, later ones Berg's recursion     */
/* with accumulated, error-weighted histograms.  Bins k = 0..K-1 have lower edges              */
/* E_k = e_lo + k eps; beta_k is the slope of -ln W over bin k.                                 */
/* ------------------------------------------------------------------------------------------ */
void orc_berg_update(int32_t K, double e_lo, double eps, const uint64_t *H, double *beta,
                     double *alpha, double *g, double beta_min, double beta_max)
{
    for (int k = 0; k + 1 < K; ++k) {
        if (H[k] == 0 || H[k + 1] == 0) continue;
        double h0 = (double)H[k], h1 = (double)H[k + 1];
        double g0 = h0 * h1 / (h0 + h1);          /* statistical weight of ln(H_{k+1}/H_k) */
        double ghat = g0 / (g[k] + g0);           /* share of this iteration in the average */
        beta[k] += ghat * (log(h1) - log(h0)) / eps;
        if (beta_max > beta_min) {                /* inverse-temperature range of interest */
            if (beta[k] < beta_min) beta[k] = beta_min;
            if (beta[k] > beta_max) beta[k] = beta_max;
        }
        g[k] += g0;
    }
    if (K >= 2) beta[K - 1] = beta[K - 2];
    int lowest = -1;                              /* lowest bin with accumulated statistics */
    for (int k = 0; k < K; ++k) if (g[k] > 0.0) { lowest = k; break; }
    for (int k = 0; k < lowest; ++k) beta[k] = beta[lowest];
    alpha[K - 1] = 0.0;                           /* continuity of ln W at every bin edge */
    for (int k = K - 2; k >= 0; --k)
        alpha[k] = alpha[k + 1] + (beta[k] - beta[k + 1]) * (e_lo + (double)(k + 1) * eps);
}

/* Flatness of a histogram over the bins between the lowest and highest visited ones:
 * c_Var = sigma_H / mu_H (population sigma) and the largest |H_k - mu_H| / mu_H (Sec. 4.1). */
void orc_flatness(int32_t K, const uint64_t *H, double *cvar, double *peak, int32_t *kmin,
                  int32_t *kmax)
{
    int lo = -1, hi = -1;
    for (int k = 0; k < K; ++k) if (H[k]) { if (lo < 0) lo = k; hi = k; }
    *kmin = lo; *kmax = hi;
    if (lo < 0) { *cvar = 0; *peak = 0; return; }
    double n = hi - lo + 1, mu = 0, var = 0, mx = 0;
    for (int k = lo; k <= hi; ++k) mu += (double)H[k];
    mu /= n;
    for (int k = lo; k <= hi; ++k) {
        double d = (double)H[k] - mu;
        var += d * d;
        if (fabs(d) > mx) mx = fabs(d);
    }
    *cvar = sqrt(var / n) / mu;
    *peak = mx / mu;
}

/* ------------------------------------------------------------------------------------------ */
/* Energy gradients for parameter differentiation (not in the paper).  theta = (C_AB, C_BB,    */
/* kappa_bend, kappa_tors) for a two-letter lexicon with C_AA fixed: E is linear in each.      */
/* dE/dx (N x 3) is the analytic gradient of the same energy function.                        */
/* ------------------------------------------------------------------------------------------ */
static void add_bond_pair_grad(const double *xa, const double *xb, const double *xc,
                               const double *xd, double kappa, double *ga, double *gb,
                               double *gc, double *gd)
{
    /* term kappa (1 - u.v), u = (xb - xa)/|xb - xa|, v = (xd - xc)/|xd - xc| */
    double p[3] = {xb[0] - xa[0], xb[1] - xa[1], xb[2] - xa[2]};
    double q[3] = {xd[0] - xc[0], xd[1] - xc[1], xd[2] - xc[2]};
    double np = sqrt(dot3(p, p)), nq = sqrt(dot3(q, q));
    double u[3] = {p[0] / np, p[1] / np, p[2] / np}, v[3] = {q[0] / nq, q[1] / nq, q[2] / nq};
    double cth = dot3(u, v);
    for (int a = 0; a < 3; ++a) {
        double dp = -kappa * (v[a] - cth * u[a]) / np;   /* d term / d p */
        double dq = -kappa * (u[a] - cth * v[a]) / nq;   /* d term / d q */
        gb[a] += dp; ga[a] -= dp;
        gd[a] += dq; gc[a] -= dq;
    }
}

void orc_energy_grad(const orc_system *s, const double *pos, double *energy, double *dedx,
                     double dedtheta[4])
{
    int n = s->n_beads;
    memset(dedx, 0, sizeof(double) * 3 * (size_t)n);
    for (int t = 0; t < 4; ++t) dedtheta[t] = 0;
    *energy = orc_energy(s, pos, NULL, NULL);
    for (int c = 0; c < s->n_chains; ++c) {
        int first = s->chain_start[c], last = s->chain_start[c + 1] - 1;
        for (int i = first; i + 2 <= last; ++i) {
            double u1[3], u2[3];
            unit_bond(pos + 3 * i, pos + 3 * (i + 1), u1);
            unit_bond(pos + 3 * (i + 1), pos + 3 * (i + 2), u2);
            dedtheta[2] += 1.0 - dot3(u1, u2);
            add_bond_pair_grad(pos + 3 * i, pos + 3 * (i + 1), pos + 3 * (i + 1), pos + 3 * (i + 2),
                               s->k_bend, dedx + 3 * i, dedx + 3 * (i + 1), dedx + 3 * (i + 1),
                               dedx + 3 * (i + 2));
        }
        for (int i = first; i + 3 <= last; ++i) {
            double u1[3], u3[3];
            unit_bond(pos + 3 * i, pos + 3 * (i + 1), u1);
            unit_bond(pos + 3 * (i + 2), pos + 3 * (i + 3), u3);
            dedtheta[3] += 1.0 - dot3(u1, u3);
            add_bond_pair_grad(pos + 3 * i, pos + 3 * (i + 1), pos + 3 * (i + 2), pos + 3 * (i + 3),
                               s->k_tors, dedx + 3 * i, dedx + 3 * (i + 1), dedx + 3 * (i + 2),
                               dedx + 3 * (i + 3));
        }
    }
    for (int i = 0; i < n; ++i) {
        int ci = chain_of(s, i);
        for (int j = i + 1; j < n; ++j) {
            int cj = chain_of(s, j);
            if (ci == cj && j == i + 1) continue;
            double d[3];
            separation(s, pos + 3 * i, pos + 3 * j, d);
            double r2 = dot3(d, d);
            double inv6 = 1.0 / (r2 * r2 * r2);
            double kappa = (ci == cj) ? s->k_intra : s->k_inter;
            double c = s->c_lj[s->type[i] * s->n_types + s->type[j]];
            int ti = s->type[i], tj = s->type[j];
            if (ti != tj) dedtheta[0] += -kappa * inv6;          /* C_AB pair */
            else if (ti == 1) dedtheta[1] += -kappa * inv6;      /* C_BB pair */
            /* d/dr2 of kappa (r2^-6 - c r2^-3) = kappa (-6 r2^-7 + 3 c r2^-4) */
            double dr2 = kappa * (-6.0 * inv6 * inv6 / r2 + 3.0 * c * inv6 / r2);
            for (int a = 0; a < 3; ++a) {
                double f = dr2 * 2.0 * d[a];
                dedx[3 * i + a] += f;
                dedx[3 * j + a] -= f;
            }
        }
    }
}

/* Full energy of n_cfg configurations stored back to back (n_cfg x N x 3). */
void orc_energy_many(const orc_system *s, int64_t n_cfg, const double *pos, double *out)
{
    for (int64_t i = 0; i < n_cfg; ++i) out[i] = orc_energy(s, pos + (size_t)i * 3 * s->n_beads, NULL, NULL);
}
