/*
 * Fixed-point multiprecision engine for the two-step Lax-Wendroff scheme
 * (TEST INFRASTRUCTURE: the oracle the GPU path is checked against; it shares
 * no code with the library).
 *
 * Numbers are signed fixed point with FRAC = 384 fraction bits and 64 integer
 * bits: NL = 7 little-endian 64-bit limbs in two's complement.  Additions and
 * subtractions are exact; a product is rounded once, to nearest with ties
 * away from zero (so negation commutes with rounding).  Any integer-part
 * overflow aborts the run with an error code rather than wrapping.
 *
 * The update is the paper's (lw1)/(lw2) (Sec. "Teukolsky Code") written for
 * the complex pair (Phi, Pi): D = diag(b, b, -b, -b) acts as +b on Phi and -b
 * on Pi, S_Phi = Pi, S_Pi = -K d_r* Phi + W Lth Phi + C0 Phi - Ct Pi, with the
 * angular operator Lth = D2 + cot(theta) D1 + V(theta) built from centred
 * stencils of reach R and reflected ghost rows of sign (-1)^|m|.  At the
 * half point the stage-1 source uses the neighbour average of u and the
 * neighbour difference over dr*; stage 2 does the same with the half-step
 * values.  Radial boundary nodes are held at zero.
 *
 * Array layouts (row-major, every entry NL limbs):
 *   u         [4][nth][nr]        Phi_R, Phi_I, Pi_R, Pi_I; overwritten
 *   coef_half [nth][nr-1][8]      b, W, K_R, K_I, Ct_R, Ct_I, C0_R, C0_I at r*_{i+1/2}
 *   coef_full [nth][nr][8]        the same at r*_i
 *   cot, V    [nth]
 *   d1, d2    [2R+1]              stencil weights already divided by dtheta, dtheta^2
 *   scal      [2]                 inv_h = 1/dr*, dt
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NL 7
#define FRAC 384

typedef struct { uint64_t w[NL]; } fx;
typedef struct { fx re, im; } cx;
typedef unsigned __int128 u128;

static int g_overflow;

static void fx_add(fx *r, const fx *a, const fx *b) {
    u128 c = 0;
    for (int k = 0; k < NL; k++) {
        c += (u128)a->w[k] + b->w[k];
        r->w[k] = (uint64_t)c;
        c >>= 64;
    }
}

static void fx_neg(fx *r, const fx *a) {
    u128 c = 1;
    for (int k = 0; k < NL; k++) {
        c += (u128)(~a->w[k]);
        r->w[k] = (uint64_t)c;
        c >>= 64;
    }
}

static void fx_sub(fx *r, const fx *a, const fx *b) {
    fx nb;
    fx_neg(&nb, b);
    fx_add(r, a, &nb);
}

static int fx_isneg(const fx *a) { return (int64_t)a->w[NL - 1] < 0; }

static void fx_mul(fx *r, const fx *a, const fx *b) {
    fx ma, mb;
    int neg = 0;
    if (fx_isneg(a)) { fx_neg(&ma, a); neg ^= 1; } else { ma = *a; }
    if (fx_isneg(b)) { fx_neg(&mb, b); neg ^= 1; } else { mb = *b; }
    uint64_t p[2 * NL + 1];
    memset(p, 0, sizeof p);
    for (int i = 0; i < NL; i++) {
        if (!ma.w[i]) continue;
        u128 carry = 0;
        for (int j = 0; j < NL; j++) {
            u128 t = (u128)ma.w[i] * mb.w[j] + p[i + j] + carry;
            p[i + j] = (uint64_t)t;
            carry = t >> 64;
        }
        p[i + NL] = (uint64_t)carry;
    }
    /* round: add 2^(FRAC-1), then drop FRAC bits (FRAC is a whole number of limbs) */
    u128 c = (u128)p[FRAC / 64 - 1] + ((uint64_t)1 << 63);
    p[FRAC / 64 - 1] = (uint64_t)c;
    c >>= 64;
    for (int k = FRAC / 64; k < 2 * NL && c; k++) {
        c += p[k];
        p[k] = (uint64_t)c;
        c >>= 64;
    }
    fx out;
    for (int k = 0; k < NL; k++) out.w[k] = p[k + FRAC / 64];
    for (int k = NL + FRAC / 64; k < 2 * NL; k++)
        if (p[k]) __atomic_store_n(&g_overflow, 1, __ATOMIC_RELAXED);
    if (fx_isneg(&out)) __atomic_store_n(&g_overflow, 1, __ATOMIC_RELAXED);
    if (neg) fx_neg(r, &out); else *r = out;
}

static void cx_add(cx *r, const cx *a, const cx *b) { fx_add(&r->re, &a->re, &b->re); fx_add(&r->im, &a->im, &b->im); }
static void cx_sub(cx *r, const cx *a, const cx *b) { fx_sub(&r->re, &a->re, &b->re); fx_sub(&r->im, &a->im, &b->im); }
static void cx_rmul(cx *r, const fx *x, const cx *a) { fx_mul(&r->re, x, &a->re); fx_mul(&r->im, x, &a->im); }
static void cx_neg(cx *r, const cx *a) { fx_neg(&r->re, &a->re); fx_neg(&r->im, &a->im); }
static void cx_mul(cx *r, const fx *zr, const fx *zi, const cx *a) {
    fx t1, t2, re, im;
    fx_mul(&t1, zr, &a->re);
    fx_mul(&t2, zi, &a->im);
    fx_sub(&re, &t1, &t2);
    fx_mul(&t1, zr, &a->im);
    fx_mul(&t2, zi, &a->re);
    fx_add(&im, &t1, &t2);
    r->re = re;
    r->im = im;
}

typedef struct {
    int nr, nth, R, parity;
    const fx *coef_half, *coef_full, *cot, *V, *d1, *d2;
    fx inv_h, dt, hdt, half;
} ctx_t;

/* Lth of column col (nth complex entries) at row j */
static void theta_op(cx *out, const cx *col, int j, const ctx_t *c) {
    cx s2, s1, v, t;
    memset(&s2, 0, sizeof s2);
    memset(&s1, 0, sizeof s1);
    for (int k = -c->R; k <= c->R; k++) {
        int q = j + k, neg = 0;
        if (q < 0) { q = -1 - q; neg = c->parity < 0; }
        else if (q >= c->nth) { q = 2 * c->nth - 1 - q; neg = c->parity < 0; }
        if (neg) cx_neg(&v, &col[q]); else v = col[q];
        cx_rmul(&t, &c->d2[k + c->R], &v);
        cx_add(&s2, &s2, &t);
        cx_rmul(&t, &c->d1[k + c->R], &v);
        cx_add(&s1, &s1, &t);
    }
    cx_rmul(&t, &c->cot[j], &s1);
    cx_add(&s2, &s2, &t);
    cx_rmul(&t, &c->V[j], &col[j]);
    cx_add(out, &s2, &t);
}

/* S_Pi = -K dphi + W lth + C0 phiv - Ct piv, with coefficient block cf[8] */
static void source_pi(cx *out, const fx *cf, const cx *dphi, const cx *lth, const cx *phiv, const cx *piv) {
    cx t, acc;
    cx_mul(&t, &cf[2], &cf[3], dphi);
    cx_neg(&acc, &t);
    cx_rmul(&t, &cf[1], lth);
    cx_add(&acc, &acc, &t);
    cx_mul(&t, &cf[6], &cf[7], phiv);
    cx_add(&acc, &acc, &t);
    cx_mul(&t, &cf[4], &cf[5], piv);
    cx_sub(out, &acc, &t);
}

/* state is internal column-major: phi[i*nth + j] */
static void lw_step(const ctx_t *c, const cx *phi, const cx *pi, cx *phih, cx *pih, cx *nphi, cx *npi) {
    const int nr = c->nr, nth = c->nth;
    /* (lw1) half step at r*_{i+1/2} */
#pragma omp parallel
    {
        cx *bar_phi = malloc(sizeof(cx) * nth), *bar_pi = malloc(sizeof(cx) * nth);
#pragma omp for schedule(static)
        for (int i = 0; i < nr - 1; i++) {
            const cx *p0 = phi + (size_t)i * nth, *p1 = phi + (size_t)(i + 1) * nth;
            const cx *q0 = pi + (size_t)i * nth, *q1 = pi + (size_t)(i + 1) * nth;
            cx t;
            for (int j = 0; j < nth; j++) {
                cx_add(&t, &p1[j], &p0[j]); cx_rmul(&bar_phi[j], &c->half, &t);
                cx_add(&t, &q1[j], &q0[j]); cx_rmul(&bar_pi[j], &c->half, &t);
            }
            for (int j = 0; j < nth; j++) {
                const fx *cf = c->coef_half + ((size_t)j * (nr - 1) + i) * 8;
                cx dphi, dpi, lth, spi, br, u;
                cx_sub(&t, &p1[j], &p0[j]); cx_rmul(&dphi, &c->inv_h, &t);
                cx_sub(&t, &q1[j], &q0[j]); cx_rmul(&dpi, &c->inv_h, &t);
                theta_op(&lth, bar_phi, j, c);
                source_pi(&spi, cf, &dphi, &lth, &bar_phi[j], &bar_pi[j]);
                /* Phi: bracket = b dphi - S_Phi */
                cx_rmul(&br, &cf[0], &dphi);
                cx_sub(&br, &br, &bar_pi[j]);
                cx_rmul(&u, &c->hdt, &br);
                cx_sub(&phih[(size_t)i * nth + j], &bar_phi[j], &u);
                /* Pi: bracket = -b dpi - S_Pi */
                cx_rmul(&br, &cf[0], &dpi);
                cx_neg(&br, &br);
                cx_sub(&br, &br, &spi);
                cx_rmul(&u, &c->hdt, &br);
                cx_sub(&pih[(size_t)i * nth + j], &bar_pi[j], &u);
            }
        }
        /* (lw2) full step at interior r*_i */
#pragma omp for schedule(static)
        for (int i = 1; i < nr - 1; i++) {
            const cx *p0 = phih + (size_t)(i - 1) * nth, *p1 = phih + (size_t)i * nth;
            const cx *q0 = pih + (size_t)(i - 1) * nth, *q1 = pih + (size_t)i * nth;
            cx t;
            for (int j = 0; j < nth; j++) {
                cx_add(&t, &p1[j], &p0[j]); cx_rmul(&bar_phi[j], &c->half, &t);
                cx_add(&t, &q1[j], &q0[j]); cx_rmul(&bar_pi[j], &c->half, &t);
            }
            for (int j = 0; j < nth; j++) {
                const fx *cf = c->coef_full + ((size_t)j * nr + i) * 8;
                cx dphi, dpi, lth, spi, br, u;
                cx_sub(&t, &p1[j], &p0[j]); cx_rmul(&dphi, &c->inv_h, &t);
                cx_sub(&t, &q1[j], &q0[j]); cx_rmul(&dpi, &c->inv_h, &t);
                theta_op(&lth, bar_phi, j, c);
                source_pi(&spi, cf, &dphi, &lth, &bar_phi[j], &bar_pi[j]);
                cx_rmul(&br, &cf[0], &dphi);
                cx_sub(&br, &br, &bar_pi[j]);
                cx_rmul(&u, &c->dt, &br);
                cx_sub(&nphi[(size_t)i * nth + j], &phi[(size_t)i * nth + j], &u);
                cx_rmul(&br, &cf[0], &dpi);
                cx_neg(&br, &br);
                cx_sub(&br, &br, &spi);
                cx_rmul(&u, &c->dt, &br);
                cx_sub(&npi[(size_t)i * nth + j], &pi[(size_t)i * nth + j], &u);
            }
        }
        free(bar_phi);
        free(bar_pi);
    }
    memset(&nphi[0], 0, sizeof(cx) * nth);
    memset(&npi[0], 0, sizeof(cx) * nth);
    memset(&nphi[(size_t)(nr - 1) * nth], 0, sizeof(cx) * nth);
    memset(&npi[(size_t)(nr - 1) * nth], 0, sizeof(cx) * nth);
}

/* Threads of the parallel loops (n > 0; the OpenMP runtime reads
 * OMP_NUM_THREADS only once); returns the count now in effect. */
int oracle_set_threads(int n) {
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}

int oracle_fx_limbs(void) { return NL; }
int oracle_fx_frac_bits(void) { return FRAC; }

/* Returns 0 on success, 1 on fixed-point overflow, 2 on bad arguments, 3 on allocation failure. */
int oracle_lw_run(int nr, int nth, long nsteps, int reach, int parity,
                  const uint64_t *coef_half, const uint64_t *coef_full,
                  const uint64_t *cot, const uint64_t *V,
                  const uint64_t *d1, const uint64_t *d2,
                  const uint64_t *scal, uint64_t *u) {
    if (nr < 3 || nth < 1 || nsteps < 0 || reach < 1 || nth < reach) return 2;
    ctx_t c;
    c.nr = nr; c.nth = nth; c.R = reach; c.parity = parity;
    c.coef_half = (const fx *)coef_half; c.coef_full = (const fx *)coef_full;
    c.cot = (const fx *)cot; c.V = (const fx *)V;
    c.d1 = (const fx *)d1; c.d2 = (const fx *)d2;
    c.inv_h = ((const fx *)scal)[0];
    c.dt = ((const fx *)scal)[1];
    memset(&c.half, 0, sizeof c.half);
    c.half.w[FRAC / 64 - 1] = (uint64_t)1 << 63;           /* 1/2 */
    fx_mul(&c.hdt, &c.half, &c.dt);
    size_t n = (size_t)nr * nth;
    cx *phi = malloc(sizeof(cx) * n), *pi = malloc(sizeof(cx) * n);
    cx *nphi = malloc(sizeof(cx) * n), *npi = malloc(sizeof(cx) * n);
    cx *phih = malloc(sizeof(cx) * n), *pih = malloc(sizeof(cx) * n);
    if (!phi || !pi || !nphi || !npi || !phih || !pih) {
        free(phi); free(pi); free(nphi); free(npi); free(phih); free(pih);
        return 3;
    }
    const fx *U = (const fx *)u;
    for (int j = 0; j < nth; j++)
        for (int i = 0; i < nr; i++) {
            size_t src = (size_t)j * nr + i, dst = (size_t)i * nth + j;
            phi[dst].re = U[0 * n + src];
            phi[dst].im = U[1 * n + src];
            pi[dst].re = U[2 * n + src];
            pi[dst].im = U[3 * n + src];
        }
    g_overflow = 0;
    for (long s = 0; s < nsteps && !g_overflow; s++) {
        lw_step(&c, phi, pi, phih, pih, nphi, npi);
        cx *t = phi; phi = nphi; nphi = t;
        t = pi; pi = npi; npi = t;
    }
    fx *Uo = (fx *)u;
    for (int j = 0; j < nth; j++)
        for (int i = 0; i < nr; i++) {
            size_t dst = (size_t)j * nr + i, src = (size_t)i * nth + j;
            Uo[0 * n + dst] = phi[src].re;
            Uo[1 * n + dst] = phi[src].im;
            Uo[2 * n + dst] = pi[src].re;
            Uo[3 * n + dst] = pi[src].im;
        }
    free(phi); free(pi); free(nphi); free(npi); free(phih); free(pih);
    return g_overflow ? 1 : 0;
}
