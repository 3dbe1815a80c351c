/*
 * oracle.c -- FP64 sequential reference for parallel-in-sequence MCMC.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only tests/, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no source, header, table or helper with the
 * HIP library.  Plain loops, no vectorisation intrinsics, built with
 * -O2 -fno-fast-math.
 *
 * What it computes (every function cites the passage it follows):
 *   - target log-densities, gradients, Hessians and parameter derivatives;
 *   - MALA / ULA transitions as the paper's MALA function defines them
 *     (Sec. 3.2): proposal, Metropolis ratio with the Langevin proposal
 *     density, gate g~ = log(alpha) - log(u), accept iff g~ > 0;
 *   - HMC with leapfrog integration (Sec. 3.3 eq. for the leapfrog step,
 *     Appendix A.2 algorithm "HMC Step with Parallel Leapfrog", with its
 *     accept test read as the standard Metropolis test log U < H0 - HL);
 *   - one whole HMC transition as the step f_t of a chain (Sec. 3.3,
 *     parallel HMC across the sequence), optionally with a diagonal mass
 *     matrix, with its Jacobian under the frozen or the relaxed gate;
 *   - the Jacobians the Newton update needs (Sec. 2 eq. 2; MALA gate via the
 *     stop-gradient relaxation, Sec. 3.2; leapfrog block form, Sec. 3.3 and
 *     Appendix A.3);
 *   - sequential solves of the linearised recursion (Sec. 2 eq. 3; quasi-DEER
 *     eq. 4; block quasi-DEER, Appendix A.3);
 *   - forward (tangent) and reverse (adjoint) derivatives of a trajectory
 *     functional through the sequential chain with the accept pattern frozen.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_GAUSSIAN = 0, ORC_BANANA = 1, ORC_LOGREG = 2, ORC_FUNNEL = 3 };

typedef struct {
    int kind;
    int dim;
    const double *mean; /* gaussian: [D]          */
    const double *prec; /* gaussian: [D*D]        */
    const double *X;    /* logreg:   [N*D]        */
    const double *y;    /* logreg:   [N] in {0,1} */
    int n;              /* logreg:   N            */
    double prior_var;   /* logreg:   prior N(0, prior_var I) */
    double theta;       /* funnel:   neck log-scale */
} orc_target;

#define MAXD 1024

static double softplus(double z) { return z > 0 ? z + log1p(exp(-z)) : log1p(exp(z)); }
static double sigmoid(double z) { return z >= 0 ? 1.0 / (1.0 + exp(-z)) : exp(z) / (1.0 + exp(z)); }

/* ---------------------------------------------------------------- targets */

/* log p(x) up to an additive constant. */
double orc_logp(const orc_target *tg, const double *x)
{
    int D = tg->dim;
    switch (tg->kind) {
    case ORC_GAUSSIAN: { /* -1/2 (x-mu)^T P (x-mu) */
        double s = 0;
        for (int i = 0; i < D; i++)
            for (int j = 0; j < D; j++)
                s += (x[i] - tg->mean[i]) * tg->prec[i * D + j] * (x[j] - tg->mean[j]);
        return -0.5 * s;
    }
    case ORC_BANANA: { /* -x1^2/2 - (x2 - x1^2)^2/2 */
        double a = x[1] - x[0] * x[0];
        return -0.5 * x[0] * x[0] - 0.5 * a * a;
    }
    case ORC_LOGREG: { /* sum_n [y z - log(1+e^z)] - |w|^2/(2 s2), z = X w */
        double s = 0;
        for (int n = 0; n < tg->n; n++) {
            double z = 0;
            for (int d = 0; d < D; d++) z += tg->X[n * D + d] * x[d];
            s += tg->y[n] * z - softplus(z);
        }
        double r = 0;
        for (int d = 0; d < D; d++) r += x[d] * x[d];
        return s - 0.5 * r / tg->prior_var;
    }
    case ORC_FUNNEL: { /* x1 ~ N(0, e^{2 theta}); x_d | x1 ~ N(0, e^{x1}) */
        double q = 0;
        for (int d = 1; d < D; d++) q += x[d] * x[d];
        return -0.5 * x[0] * x[0] * exp(-2 * tg->theta) - tg->theta - 0.5 * exp(-x[0]) * q
               - 0.5 * (D - 1) * x[0];
    }
    }
    return NAN;
}

void orc_grad(const orc_target *tg, const double *x, double *g)
{
    int D = tg->dim;
    switch (tg->kind) {
    case ORC_GAUSSIAN:
        for (int i = 0; i < D; i++) {
            double s = 0;
            for (int j = 0; j < D; j++) s += tg->prec[i * D + j] * (x[j] - tg->mean[j]);
            g[i] = -s;
        }
        return;
    case ORC_BANANA: {
        double a = x[1] - x[0] * x[0];
        g[0] = -x[0] + 2 * x[0] * a;
        g[1] = -a;
        return;
    }
    case ORC_LOGREG:
        for (int d = 0; d < D; d++) g[d] = -x[d] / tg->prior_var;
        for (int n = 0; n < tg->n; n++) {
            double z = 0;
            for (int d = 0; d < D; d++) z += tg->X[n * D + d] * x[d];
            double r = tg->y[n] - sigmoid(z);
            for (int d = 0; d < D; d++) g[d] += r * tg->X[n * D + d];
        }
        return;
    case ORC_FUNNEL: {
        double q = 0, e = exp(-x[0]);
        for (int d = 1; d < D; d++) q += x[d] * x[d];
        g[0] = -x[0] * exp(-2 * tg->theta) + 0.5 * e * q - 0.5 * (D - 1);
        for (int d = 1; d < D; d++) g[d] = -e * x[d];
        return;
    }
    }
}

/* Dense Hessian of log p, row-major D x D. */
void orc_hess(const orc_target *tg, const double *x, double *H)
{
    int D = tg->dim;
    memset(H, 0, sizeof(double) * D * D);
    switch (tg->kind) {
    case ORC_GAUSSIAN:
        for (int i = 0; i < D * D; i++) H[i] = -tg->prec[i];
        return;
    case ORC_BANANA:
        H[0] = -1 + 2 * (x[1] - x[0] * x[0]) - 4 * x[0] * x[0];
        H[1] = H[2] = 2 * x[0];
        H[3] = -1;
        return;
    case ORC_LOGREG:
        for (int d = 0; d < D; d++) H[d * D + d] = -1.0 / tg->prior_var;
        for (int n = 0; n < tg->n; n++) {
            const double *xn = tg->X + (size_t)n * D;
            double z = 0;
            for (int d = 0; d < D; d++) z += xn[d] * x[d];
            double s = sigmoid(z), w = s * (1 - s);
            for (int i = 0; i < D; i++)
                for (int j = 0; j < D; j++) H[i * D + j] -= w * xn[i] * xn[j];
        }
        return;
    case ORC_FUNNEL: {
        double q = 0, e = exp(-x[0]);
        for (int d = 1; d < D; d++) q += x[d] * x[d];
        H[0] = -exp(-2 * tg->theta) - 0.5 * e * q;
        for (int d = 1; d < D; d++) {
            H[d] = H[d * D] = e * x[d];
            H[d * D + d] = -e;
        }
        return;
    }
    }
}

/* d/dtheta of grad log p (only the funnel depends on theta). */
void orc_dgrad_dtheta(const orc_target *tg, const double *x, double *out)
{
    for (int d = 0; d < tg->dim; d++) out[d] = 0;
    if (tg->kind == ORC_FUNNEL) out[0] = 2 * x[0] * exp(-2 * tg->theta);
}

/* d/dtheta of log p (only the funnel depends on theta). */
double orc_dlogp_dtheta(const orc_target *tg, const double *x)
{
    if (tg->kind == ORC_FUNNEL) return x[0] * x[0] * exp(-2 * tg->theta) - 1;
    return 0;
}

/* ------------------------------------------------------------------ MALA */

/* log q(a | b) for the Langevin proposal N(b + eps grad log p(b), 2 eps I),
 * without its normalising constant (it cancels in the ratio). */
static double log_q(int D, const double *a, const double *b, const double *grad_b, double eps)
{
    double s = 0;
    for (int d = 0; d < D; d++) {
        double r = a[d] - b[d] - eps * grad_b[d];
        s += r * r;
    }
    return -s / (4 * eps);
}

/*
 * One MALA transition f_t(x) = MALA(x, {xi_t, u_t}) (Sec. 3.2, the MALA
 * function).  Proposal x~ = x + eps grad log p(x) + sqrt(2 eps) xi; acceptance
 * alpha = min{1, p(x~) q(x | x~) / (p(x) q(x~ | x))}; gate g~ = log alpha - log u;
 * the forward pass keeps x~ iff g~ > 0 (the indicator of the stop-gradient
 * construction).  ULA (ula != 0) always keeps x~.
 * force: -1 = use the computed decision, 0/1 = impose it.
 * Writes x_next; returns the decision; *gt = g~, *ell = log of the ratio.
 */
int orc_mala_step(const orc_target *tg, double eps, int ula, const double *x, const double *xi,
                  double u, int force, double *x_next, double *gt, double *ell, double *xprop)
{
    int D = tg->dim;
    double g[MAXD], xt[MAXD], gt_[MAXD];
    orc_grad(tg, x, g);
    double c = sqrt(2 * eps);
    for (int d = 0; d < D; d++) xt[d] = x[d] + eps * g[d] + c * xi[d];
    if (xprop)
        for (int d = 0; d < D; d++) xprop[d] = xt[d];
    if (ula) {
        for (int d = 0; d < D; d++) x_next[d] = xt[d];
        if (gt) *gt = INFINITY;
        if (ell) *ell = 0;
        return 1;
    }
    orc_grad(tg, xt, gt_);
    double l = orc_logp(tg, xt) - orc_logp(tg, x) + log_q(D, x, xt, gt_, eps) - log_q(D, xt, x, g, eps);
    double log_alpha = l < 0 ? l : 0;
    double gg = log_alpha - log(u);
    /* a NaN log ratio (a diverged proposal, inf - inf) rejects */
    int acc = gg > 0 && l == l;
    if (force == 0 || force == 1) acc = force;
    for (int d = 0; d < D; d++) x_next[d] = acc ? xt[d] : x[d];
    if (gt) *gt = gg;
    if (ell) *ell = l;
    return acc;
}

/*
 * Sequential MALA/ULA chain s_t = f_t(s_{t-1}), t = 1..T (Sec. 2, the
 * recursion evaluated step by step).  xi: [T*D], u: [T].  force: NULL or [T]
 * with entries -1 (free), 0 or 1 (impose the decision at that step).
 * Outputs: states [T*D], accept [T], gtilde [T] (each may be NULL except states).
 * Returns the number of accepted steps.
 */
long orc_mala_chain(const orc_target *tg, double eps, int ula, long T, const double *x0,
                    const double *xi, const double *u, const int8_t *force, double *states,
                    int8_t *accept, double *gtilde)
{
    int D = tg->dim;
    double x[MAXD];
    long nacc = 0;
    for (int d = 0; d < D; d++) x[d] = x0[d];
    for (long t = 0; t < T; t++) {
        double gg;
        int f = force ? force[t] : -1;
        int a = orc_mala_step(tg, eps, ula, x, xi + t * D, ula ? 0.5 : u[t], f, states + t * D, &gg,
                              NULL, NULL);
        nacc += a;
        if (accept) accept[t] = (int8_t)a;
        if (gtilde) gtilde[t] = gg;
        for (int d = 0; d < D; d++) x[d] = states[t * D + d];
    }
    return nacc;
}

/*
 * Jacobian J = df_t/dx of one MALA transition at x, and F = f_t(x).
 * gate 0 (frozen): J = a (I + eps H(x)) + (1 - a) I, the accept decision a
 *   treated as a constant.
 * gate 1 (surrogate): the stop-gradient gate of Sec. 3.2,
 *   g = sigma(g~) + sg(1(g~>0) - sigma(g~)): forward value a, derivative
 *   sigma'(g~) dg~/dx, so J gains the rank-one term
 *   sigma(g~)(1 - sigma(g~)) (x~ - x) (d g~/dx)^T,
 *   with d g~/dx = 1(l < 0) dl/dx, l the log Metropolis ratio.
 *   Derivation of dl/dx (x~ = x + eps g + c xi, g = grad log p(x),
 *   g' = grad log p(x~), M = dx~/dx = I + eps H(x), w = x - x~ - eps g'):
 *     l = log p(x~) - log p(x) - |w|^2/(4 eps) + |x~ - x - eps g|^2/(4 eps),
 *     the last term equals |xi|^2/2 and does not depend on x;
 *     dw/dx = -eps H(x) - eps H(x~) M, hence
 *     dl/dx = M g' - g + (H(x) w + M H(x~) w) / 2.
 * ULA: J = I + eps H(x).
 * force as in orc_mala_step.  Returns the decision.
 */
int orc_mala_jac(const orc_target *tg, double eps, int ula, int gate, const double *x,
                 const double *xi, double u, int force, double *F, double *J)
{
    int D = tg->dim;
    static double H[MAXD * MAXD], Ht[MAXD * MAXD];
    double xt[MAXD], g[MAXD], gp[MAXD], w[MAXD], hw[MAXD], htw[MAXD], mhtw[MAXD], dl[MAXD];
    double gg, l;
    int a = orc_mala_step(tg, eps, ula, x, xi, u, force, F, &gg, &l, xt);
    orc_hess(tg, x, H);
    for (int i = 0; i < D; i++)
        for (int j = 0; j < D; j++)
            J[i * D + j] = (i == j ? 1.0 : 0.0) + (a ? eps * H[i * D + j] : 0.0);
    if (ula || gate == 0) return a;
    /* surrogate rank-one term */
    if (!(l < 0)) return a; /* d g~/dx = 0 where the min picks the constant 0 */
    orc_grad(tg, x, g);
    orc_grad(tg, xt, gp);
    orc_hess(tg, xt, Ht);
    for (int d = 0; d < D; d++) w[d] = x[d] - xt[d] - eps * gp[d];
    for (int i = 0; i < D; i++) {
        double s1 = 0, s2 = 0;
        for (int j = 0; j < D; j++) {
            s1 += H[i * D + j] * w[j];
            s2 += Ht[i * D + j] * w[j];
        }
        hw[i] = s1;
        htw[i] = s2;
    }
    /* M v = v + eps H(x) v */
    for (int i = 0; i < D; i++) {
        double s = 0, s2 = 0;
        for (int j = 0; j < D; j++) {
            s += H[i * D + j] * gp[j];
            s2 += H[i * D + j] * htw[j];
        }
        mhtw[i] = htw[i] + eps * s2;
        dl[i] = (gp[i] + eps * s) - g[i] + 0.5 * hw[i] + 0.5 * mhtw[i];
    }
    double sg = 1.0 / (1.0 + exp(-gg));
    double c = sg * (1 - sg);
    for (int i = 0; i < D; i++)
        for (int j = 0; j < D; j++) J[i * D + j] += c * (xt[i] - x[i]) * dl[j];
    return a;
}

/* The sigma-smoothed MALA step (gate sigma(g~) used in the forward pass too);
 * used only to pin the surrogate Jacobian by finite differences. */
void orc_mala_smoothed_step(const orc_target *tg, double eps, const double *x, const double *xi,
                            double u, double *out)
{
    int D = tg->dim;
    double xt[MAXD], xn[MAXD], gg;
    orc_mala_step(tg, eps, 0, x, xi, u, -1, xn, &gg, NULL, xt);
    double s = 1.0 / (1.0 + exp(-gg));
    for (int d = 0; d < D; d++) out[d] = s * xt[d] + (1 - s) * x[d];
}

/* ------------------------------------------------------------- leapfrog */

/* One leapfrog step of Sec. 3.3: x' = x + eps v; v' = v + eps grad log p(x').
 * s = [x, v] (2D).  If J != NULL also writes the 2D x 2D Jacobian
 * [[I, eps I], [eps H(x'), I + eps^2 H(x')]] (Sec. 3.3, Appendix A.3). */
void orc_leapfrog_step(const orc_target *tg, double eps, const double *s, double *out, double *J)
{
    int D = tg->dim;
    double g[MAXD];
    for (int d = 0; d < D; d++) out[d] = s[d] + eps * s[D + d];
    orc_grad(tg, out, g);
    for (int d = 0; d < D; d++) out[D + d] = s[D + d] + eps * g[d];
    if (J) {
        static double H[MAXD * MAXD];
        int M = 2 * D;
        orc_hess(tg, out, H);
        for (int i = 0; i < M * M; i++) J[i] = 0;
        for (int i = 0; i < D; i++) {
            J[i * M + i] = 1;
            J[i * M + D + i] = eps;
            for (int j = 0; j < D; j++) {
                J[(D + i) * M + j] = eps * H[i * D + j];
                J[(D + i) * M + D + j] = (i == j ? 1.0 : 0.0) + eps * eps * H[i * D + j];
            }
        }
    }
}

/*
 * HMC with a fixed number L of leapfrog steps (Appendix A.2 algorithm), run
 * sequentially over n_prop proposals.  For proposal p: v0 = momenta[p];
 * H0 = v0.v0/2 - log p(x0); half step v0 += eps/2 grad log p(x0); L leapfrog
 * steps; reverse half step vL -= eps/2 grad log p(xL); HL = vL.vL/2 - log p(xL);
 * accept iff log U_p < H0 - HL (standard Metropolis test; the printed test is
 * garbled and is read this way).
 * Outputs: chain [(n_prop+1)*D] (row 0 = x0); accept [n_prop]; logr [n_prop]
 * = (H0 - HL) - log U; s0 [n_prop*2D] = the leapfrog recursion's initial state
 * [x0, v after the half step]; traj [n_prop*L*2D] = s_1..s_L.  Optional ones
 * may be NULL.  force: NULL or [n_prop] of -1/0/1.
 */
long orc_hmc_chain(const orc_target *tg, double eps, int L, long n_prop, const double *x0,
                   const double *momenta, const double *U, const int8_t *force, double *chain,
                   int8_t *accept, double *logr, double *s0, double *traj)
{
    int D = tg->dim;
    double x[MAXD], s[2 * MAXD], sn[2 * MAXD], g[MAXD];
    long nacc = 0;
    for (int d = 0; d < D; d++) chain[d] = x[d] = x0[d];
    for (long p = 0; p < n_prop; p++) {
        const double *v0 = momenta + p * D;
        double kin = 0;
        for (int d = 0; d < D; d++) kin += v0[d] * v0[d];
        double H0 = 0.5 * kin - orc_logp(tg, x);
        orc_grad(tg, x, g);
        for (int d = 0; d < D; d++) {
            s[d] = x[d];
            s[D + d] = v0[d] + 0.5 * eps * g[d];
        }
        if (s0)
            for (int d = 0; d < 2 * D; d++) s0[p * 2 * D + d] = s[d];
        for (int l = 0; l < L; l++) {
            orc_leapfrog_step(tg, eps, s, sn, NULL);
            memcpy(s, sn, sizeof(double) * 2 * D);
            if (traj)
                for (int d = 0; d < 2 * D; d++) traj[(p * L + l) * 2 * D + d] = s[d];
        }
        orc_grad(tg, s, g);
        kin = 0;
        for (int d = 0; d < D; d++) {
            double v = s[D + d] - 0.5 * eps * g[d];
            kin += v * v;
        }
        double HL = 0.5 * kin - orc_logp(tg, s);
        double lr = (H0 - HL) - log(U[p]);
        int a = lr > 0;
        if (force && (force[p] == 0 || force[p] == 1)) a = force[p];
        nacc += a;
        if (accept) accept[p] = (int8_t)a;
        if (logr) logr[p] = lr;
        if (a)
            for (int d = 0; d < D; d++) x[d] = s[d];
        for (int d = 0; d < D; d++) chain[(p + 1) * D + d] = x[d];
    }
    return nacc;
}

/* ------------------------------------- HMC across the sequence (Sec. 3.3) */

/*
 * One whole HMC transition x_t = f_t(x_{t-1}) with its sequential leapfrog
 * integrator, the map that Sec. 3.3 ("Parallel HMC with Sequential Leapfrog
 * Integration") parallelises across the steps of the chain.  Momentum
 * v0 = xi / sqrt(inv_mass) (inv_mass: diagonal of M^-1, NULL = identity), so
 * xi ~ N(0, I) gives v0 ~ N(0, M); half step v = v0 + eps/2 grad log p(x);
 * L leapfrog steps x <- x + eps M^-1 v, v <- v + eps grad log p(x); reverse
 * half step v_f = v - eps/2 grad log p(x_L); energies
 * H = v.M^-1 v / 2 - log p(x) (Appendix A.2, with the accept test read as
 * the Metropolis test); log alpha = min(0, H0 - HL); gate
 * g~ = log alpha - log u; accept iff g~ > 0 (the forward value of the
 * relaxed gate of Sec. 3.2).  force as in orc_mala_step.
 * Writes x_next (and the proposal x_L to xprop, and H0 - HL to dh, when not
 * NULL); returns the decision; *gt = g~.
 */
int orc_hmc_step(const orc_target *tg, double eps, int L, const double *inv_mass, const double *x,
                 const double *xi, double u, int force, double *x_next, double *gt, double *dh,
                 double *xprop)
{
    int D = tg->dim;
    double g[MAXD], xl[MAXD], v[MAXD], v0[MAXD];
    double kin0 = 0, kinL = 0;
    for (int d = 0; d < D; d++) {
        double im = inv_mass ? inv_mass[d] : 1.0;
        v0[d] = xi[d] / sqrt(im);
        kin0 += v0[d] * im * v0[d];
    }
    double H0 = 0.5 * kin0 - orc_logp(tg, x);
    orc_grad(tg, x, g);
    for (int d = 0; d < D; d++) {
        xl[d] = x[d];
        v[d] = v0[d] + 0.5 * eps * g[d];
    }
    for (int l = 0; l < L; l++) {
        for (int d = 0; d < D; d++) xl[d] += eps * (inv_mass ? inv_mass[d] : 1.0) * v[d];
        orc_grad(tg, xl, g);
        for (int d = 0; d < D; d++) v[d] += eps * g[d];
    }
    for (int d = 0; d < D; d++) {
        double vf = v[d] - 0.5 * eps * g[d];
        kinL += vf * (inv_mass ? inv_mass[d] : 1.0) * vf;
    }
    double HL = 0.5 * kinL - orc_logp(tg, xl);
    double diff = H0 - HL;
    double log_alpha = diff < 0 ? diff : 0;
    double gg = log_alpha - log(u);
    /* a NaN energy difference (a diverged trajectory, inf - inf) rejects */
    int acc = gg > 0 && diff == diff;
    if (force == 0 || force == 1) acc = force;
    for (int d = 0; d < D; d++) x_next[d] = acc ? xl[d] : x[d];
    if (xprop)
        for (int d = 0; d < D; d++) xprop[d] = xl[d];
    if (gt) *gt = gg;
    if (dh) *dh = diff;
    return acc;
}

/* Sequential chain of HMC transitions (Sec. 2, the recursion evaluated step by
 * step).  xi: [T*D] standard normal momenta draws, u: [T]; force NULL or [T].
 * Outputs states [T*D], accept [T], gtilde [T] (the last two may be NULL).
 * Returns the number of accepted steps. */
long orc_hmc_seq_chain(const orc_target *tg, double eps, int L, const double *inv_mass, long T,
                       const double *x0, const double *xi, const double *u, const int8_t *force,
                       double *states, int8_t *accept, double *gtilde)
{
    int D = tg->dim;
    double x[MAXD];
    long nacc = 0;
    for (int d = 0; d < D; d++) x[d] = x0[d];
    for (long t = 0; t < T; t++) {
        double gg;
        int f = force ? force[t] : -1;
        int a = orc_hmc_step(tg, eps, L, inv_mass, x, xi + t * D, u[t], f, states + t * D, &gg, NULL, NULL);
        nacc += a;
        if (accept) accept[t] = (int8_t)a;
        if (gtilde) gtilde[t] = gg;
        for (int d = 0; d < D; d++) x[d] = states[t * D + d];
    }
    return nacc;
}

/*
 * Jacobian J = d x_t / d x_{t-1} of one HMC transition, dense D x D
 * (row-major), and F = f_t(x), by the chain rule through the integrator
 * written out in forward mode: with Xd = dx/dx0 and Vd = dv/dx0 (D x D),
 *   half step:  Xd = I, Vd = eps/2 H(x0);
 *   each leapfrog step: Xd <- Xd + eps M^-1 Vd, then Vd <- Vd + eps H(x) Xd
 *   at the new position (the Jacobian blocks of Sec. 3.3 eq. for the leapfrog
 *   step, with a mass matrix);
 * frozen gate (gate 0): J = a Xd_L + (1 - a) I;
 * relaxed gate (gate 1, the stop-gradient construction of Sec. 3.2 applied to
 * the HMC accept step): J gains sigma(g~)(1 - sigma(g~)) (x_L - x0) (dg~/dx0)^T
 * with dg~/dx0 = 1(H0 - HL < 0) d(H0 - HL)/dx0, where
 *   dH0/dx0 = -grad log p(x0),
 *   dHL/dx0 = Vf^T M^-1 v_f - Xd_L^T grad log p(x_L),
 *   Vf = Vd_L - eps/2 H(x_L) Xd_L  (the reverse half step).
 * Returns the decision.
 */
int orc_hmc_step_jac(const orc_target *tg, double eps, int L, const double *inv_mass, int gate,
                     const double *x, const double *xi, double u, int force, double *F, double *J)
{
    int D = tg->dim;
    static double H[MAXD * MAXD], Xd[MAXD * MAXD], Vd[MAXD * MAXD], T1[MAXD * MAXD];
    double g[MAXD], xl[MAXD], v[MAXD], g0[MAXD], dl[MAXD], vf[MAXD];
    double gg, diff;
    int a = orc_hmc_step(tg, eps, L, inv_mass, x, xi, u, force, F, &gg, &diff, NULL);
    /* forward pass again, carrying the tangents */
    orc_grad(tg, x, g0);
    orc_hess(tg, x, H);
    for (int i = 0; i < D; i++) g[i] = g0[i];
    for (int i = 0; i < D; i++) {
        xl[i] = x[i];
        v[i] = xi[i] / sqrt(inv_mass ? inv_mass[i] : 1.0) + 0.5 * eps * g0[i];
        for (int j = 0; j < D; j++) {
            Xd[i * D + j] = i == j ? 1.0 : 0.0;
            Vd[i * D + j] = 0.5 * eps * H[i * D + j];
        }
    }
    for (int l = 0; l < L; l++) {
        for (int i = 0; i < D; i++) {
            double im = inv_mass ? inv_mass[i] : 1.0;
            xl[i] += eps * im * v[i];
            for (int j = 0; j < D; j++) Xd[i * D + j] += eps * im * Vd[i * D + j];
        }
        orc_grad(tg, xl, g);
        orc_hess(tg, xl, H);
        for (int i = 0; i < D; i++) {
            v[i] += eps * g[i];
            for (int j = 0; j < D; j++) {
                double s = 0;
                for (int k = 0; k < D; k++) s += H[i * D + k] * Xd[k * D + j];
                T1[i * D + j] = s;
            }
        }
        for (int i = 0; i < D * D; i++) Vd[i] += eps * T1[i];
    }
    for (int i = 0; i < D; i++)
        for (int j = 0; j < D; j++) J[i * D + j] = a ? Xd[i * D + j] : (i == j ? 1.0 : 0.0);
    if (gate == 0 || !(diff < 0)) return a;
    /* relaxed gate: dg~/dx0 = d(H0 - HL)/dx0 where H0 - HL < 0 */
    for (int i = 0; i < D; i++) vf[i] = v[i] - 0.5 * eps * g[i];
    /* H = Hess at x_L (from the last leapfrog step; for L = 0 at x0) */
    for (int j = 0; j < D; j++) {
        double dHL = 0;
        for (int i = 0; i < D; i++) {
            double hx = 0;
            for (int k = 0; k < D; k++) hx += H[i * D + k] * Xd[k * D + j];
            double vfd = Vd[i * D + j] - 0.5 * eps * hx;
            dHL += vfd * (inv_mass ? inv_mass[i] : 1.0) * vf[i] - Xd[i * D + j] * g[i];
        }
        dl[j] = -g0[j] - dHL;
    }
    double sg = 1.0 / (1.0 + exp(-gg));
    double c = sg * (1 - sg);
    for (int i = 0; i < D; i++)
        for (int j = 0; j < D; j++) J[i * D + j] += c * (xl[i] - x[i]) * dl[j];
    return a;
}

/* The sigma-smoothed HMC transition (gate sigma(g~) in the forward pass too):
 * used only to pin the relaxed-gate Jacobian by finite differences. */
void orc_hmc_smoothed_step(const orc_target *tg, double eps, int L, const double *inv_mass, const double *x,
                           const double *xi, double u, double *out)
{
    int D = tg->dim;
    double xl[MAXD], xn[MAXD], gg;
    orc_hmc_step(tg, eps, L, inv_mass, x, xi, u, -1, xn, &gg, NULL, xl);
    double s = 1.0 / (1.0 + exp(-gg));
    for (int d = 0; d < D; d++) out[d] = s * xl[d] + (1 - s) * x[d];
}

/* --------------------------------------------- linear recursions (eq. 3) */

/* delta_t = a_t * delta_{t-1} + b_t elementwise, delta_0 = 0, for T steps of
 * D independent lanes; a, b, out: [T*D].  (quasi-DEER, eq. 4) */
void orc_linrec_diag(long T, int D, const double *a, const double *b, double *out)
{
    for (int d = 0; d < D; d++) {
        double s = 0;
        for (long t = 0; t < T; t++) {
            s = a[t * D + d] * s + b[t * D + d];
            out[t * D + d] = s;
        }
    }
}

/* delta_t = A_t delta_{t-1} + b_t with dense D x D A_t (row-major), delta_0 = 0.
 * A: [T*D*D], b, out: [T*D].  (DEER, eq. 3) */
void orc_linrec_dense(long T, int D, const double *A, const double *b, double *out)
{
    double s[MAXD], n[MAXD];
    for (int d = 0; d < D; d++) s[d] = 0;
    for (long t = 0; t < T; t++) {
        const double *At = A + (size_t)t * D * D;
        for (int i = 0; i < D; i++) {
            double v = b[t * D + i];
            for (int j = 0; j < D; j++) v += At[i * D + j] * s[j];
            n[i] = v;
        }
        for (int i = 0; i < D; i++) out[t * D + i] = s[i] = n[i];
    }
}

/* Block quasi-DEER recursion (Appendix A.3): state [p; q] (2 x D), per step
 * [p; q]_t = [[diag a, diag b], [diag c, diag d]] [p; q]_{t-1} + [e; f]_t.
 * a,b,c,d,e,f: [T*D]; outp, outq: [T*D]. */
void orc_linrec_block2(long T, int D, const double *a, const double *b, const double *c,
                       const double *d, const double *e, const double *f, double *outp,
                       double *outq)
{
    for (int k = 0; k < D; k++) {
        double p = 0, q = 0;
        for (long t = 0; t < T; t++) {
            size_t i = t * D + k;
            double pn = a[i] * p + b[i] * q + e[i];
            double qn = c[i] * p + d[i] * q + f[i];
            p = pn;
            q = qn;
            outp[i] = p;
            outq[i] = q;
        }
    }
}

/* --------------------------------- derivatives of trajectory functionals */

/*
 * Frozen-gate derivatives of one MALA step with respect to the target
 * parameter theta and the step size eps, at x with decision a:
 *   df/dtheta = a eps d(grad log p)/dtheta (x)
 *   df/deps   = a (grad log p(x) + xi / sqrt(2 eps))
 */
static void mala_dparams(const orc_target *tg, double eps, int a, const double *x, const double *xi,
                         double *dth, double *deps)
{
    int D = tg->dim;
    double g[MAXD], dg[MAXD];
    orc_grad(tg, x, g);
    orc_dgrad_dtheta(tg, x, dg);
    double c = 1.0 / sqrt(2 * eps);
    for (int d = 0; d < D; d++) {
        dth[d] = a ? eps * dg[d] : 0.0;
        deps[d] = a ? g[d] + c * xi[d] : 0.0;
    }
}

/*
 * Tangent (forward-mode) derivative of F(s_{1:T}) with respect to theta and
 * eps through the sequential chain, with every accept decision held at
 * accept[t] (frozen gate).  sdot_t = J_t sdot_{t-1} + df_t/dp, sdot_0 = 0;
 * dF/dp = sum_t dF/ds_t . sdot_t.  states: the chain [T*D]; dFds: [T*D].
 * out[0] = dF/dtheta, out[1] = dF/deps.
 */
void orc_mala_tangent(const orc_target *tg, double eps, int ula, long T, const double *x0,
                      const double *xi, const double *states, const int8_t *accept,
                      const double *dFds, double *out)
{
    int D = tg->dim;
    static double H[MAXD * MAXD];
    double st[MAXD], se[MAXD], nt[MAXD], ne[MAXD], dth[MAXD], dep[MAXD];
    double rt = 0, re = 0;
    for (int d = 0; d < D; d++) st[d] = se[d] = 0;
    for (long t = 0; t < T; t++) {
        const double *x = t ? states + (t - 1) * D : x0;
        int a = ula ? 1 : accept[t];
        orc_hess(tg, x, H);
        mala_dparams(tg, eps, a, x, xi + t * D, dth, dep);
        for (int i = 0; i < D; i++) {
            double ht = 0, he = 0;
            for (int j = 0; j < D; j++) {
                ht += H[i * D + j] * st[j];
                he += H[i * D + j] * se[j];
            }
            nt[i] = st[i] + (a ? eps * ht : 0.0) + dth[i];
            ne[i] = se[i] + (a ? eps * he : 0.0) + dep[i];
        }
        for (int i = 0; i < D; i++) {
            st[i] = nt[i];
            se[i] = ne[i];
            rt += dFds[t * D + i] * st[i];
            re += dFds[t * D + i] * se[i];
        }
    }
    out[0] = rt;
    out[1] = re;
}

/*
 * Adjoint (reverse-mode) derivative of the same quantity:
 * lambda_T = dF/ds_T, lambda_t = dF/ds_t + J_{t+1}^T lambda_{t+1};
 * dF/dp = sum_t lambda_t . df_t/dp.  Same inputs and outputs as the tangent.
 * If lambda_out != NULL the adjoint states are written there ([T*D]).
 */
void orc_mala_adjoint(const orc_target *tg, double eps, int ula, long T, const double *x0,
                      const double *xi, const double *states, const int8_t *accept,
                      const double *dFds, double *out, double *lambda_out)
{
    int D = tg->dim;
    static double H[MAXD * MAXD];
    double lam[MAXD], nl[MAXD], dth[MAXD], dep[MAXD];
    double rt = 0, re = 0;
    for (int d = 0; d < D; d++) lam[d] = 0;
    for (long t = T - 1; t >= 0; t--) {
        /* lambda_t = dF/ds_t + J_{t+1}^T lambda_{t+1}; J_{t+1} evaluated at s_t */
        if (t + 1 < T) {
            int a = ula ? 1 : accept[t + 1];
            orc_hess(tg, states + t * D, H);
            for (int j = 0; j < D; j++) {
                double v = 0;
                for (int i = 0; i < D; i++) v += H[i * D + j] * lam[i];
                nl[j] = lam[j] + (a ? eps * v : 0.0);
            }
        } else {
            for (int j = 0; j < D; j++) nl[j] = 0;
        }
        for (int j = 0; j < D; j++) lam[j] = nl[j] + dFds[t * D + j];
        if (lambda_out)
            for (int j = 0; j < D; j++) lambda_out[t * D + j] = lam[j];
        const double *x = t ? states + (t - 1) * D : x0;
        int a = ula ? 1 : accept[t];
        mala_dparams(tg, eps, a, x, xi + t * D, dth, dep);
        for (int j = 0; j < D; j++) {
            rt += lam[j] * dth[j];
            re += lam[j] * dep[j];
        }
    }
    out[0] = rt;
    out[1] = re;
}
