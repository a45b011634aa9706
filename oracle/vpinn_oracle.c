/*
 * FP64 CPU oracle of the FastVPINNs loss and its gradient.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference the HIP
 * library is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the library never does, and
 * the two share no code, headers or tables.
 *
 * Every quantity is computed in double precision, element by element, in the
 * order the paper defines it:
 *   - weak form and its quadrature (Section 2.3, the discrete variational
 *     problem and its quadrature approximation);
 *   - cell residual W_k = int_K grad u . grad v_k - f v_k (Section 2.3, the
 *     cell-wise residual) evaluated with the element loop of Section 3.1;
 *   - the premultiplied tensors G_x, G_y [N_elem][N_test][N_quad] and the
 *     forcing matrix F [N_elem][N_test] of Section 4.4 and Appendix A.2;
 *   - the bilinear map and its Jacobian of Appendix A.1 (inverse taken as the
 *     true inverse of the printed Jacobian matrix; the printed inverse swaps
 *     xi and eta in its second row);
 *   - the tanh network of Section 2.2 (the composition l o T^h o ... o T^1);
 *   - the total loss L_v + tau L_b + gamma L_s (Sections 2.3 and 4.7) with
 *     L_v = c_v sum_{e,k} R[e,k]^2, where c_v = 1/N_test follows Algorithm 3
 *     (mean over test functions, sum over elements) and c_v = 1/N_elem
 *     follows the variational-loss equation of Section 2.3;
 *   - Adam as in Kingma and Ba, Algorithm 1 (cited in Section 4.6.3).
 * Gradients are the chain rule written out by hand in reverse order.
 *
 * Readings where the paper is ambiguous:
 *   - quadrature is Gauss-Lobatto-Legendre with n points per direction;
 *   - the 1D test functions are phi_r = P_{r+1} - P_{r-1} (Legendre), r = 1..N_t;
 *     the 2D test function k = (s-1) N_t + (r-1) is phi_r(xi) phi_s(eta);
 *   - quadrature index q = j n + i with i the xi index and j the eta index;
 *   - the residual is R = eps * A - F with A[e,k] = sum_q grad u . G[e,k,q]
 *     (eps = 1 for the forward Poisson problem);
 *   - vertices are counter-clockwise and det J must be positive everywhere.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_ARG -1
#define ORC_E_MESH -2
#define ORC_E_NONFINITE -4

/* ------------------------------------------------------------------------- */
/* Legendre polynomials                                                       */
/* ------------------------------------------------------------------------- */

/* P_m(t) by Bonnet's recurrence (k+1) P_{k+1} = (2k+1) t P_k - k P_{k-1}. */
double orc_legendre(int m, double t)
{
    if (m == 0) return 1.0;
    double p0 = 1.0, p1 = t;
    for (int k = 1; k < m; ++k) {
        double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
    }
    return p1;
}

/* P'_m(t) by the derivative recurrence P'_{k+1} = P'_{k-1} + (2k+1) P_k. */
double orc_legendre_deriv(int m, double t)
{
    if (m == 0) return 0.0;
    double dm1 = 0.0, d = 1.0; /* P'_0, P'_1 */
    for (int k = 1; k < m; ++k) {
        double dn = dm1 + (2.0 * k + 1.0) * orc_legendre(k, t);
        dm1 = d;
        d = dn;
    }
    return d;
}

/* ------------------------------------------------------------------------- */
/* Gauss-Lobatto-Legendre rule on [-1, 1] (the rule Section 3.1 names)        */
/* nodes: -1, +1 and the roots of P'_{n-1}; weights 2 / (n (n-1) P_{n-1}^2).   */
/* ------------------------------------------------------------------------- */
int orc_gll(int n, double *x, double *w)
{
    if (n < 2 || n > 128 || !x || !w) return ORC_E_ARG;
    const int m = n - 1;
    x[0] = -1.0;
    x[n - 1] = 1.0;
    for (int i = 1; i < n - 1; ++i) {
        double t = -cos(M_PI * (double)i / (double)m);
        for (int it = 0; it < 100; ++it) {
            double p = orc_legendre(m, t);
            double dp = orc_legendre_deriv(m, t);
            /* Legendre's equation: (1 - t^2) P'' = 2 t P' - m (m+1) P */
            double ddp = (2.0 * t * dp - m * (m + 1.0) * p) / (1.0 - t * t);
            double dt = dp / ddp;
            t -= dt;
            if (fabs(dt) < 1e-16) break;
        }
        x[i] = t;
    }
    for (int i = 0; i < n; ++i) {
        double p = orc_legendre(m, x[i]);
        w[i] = 2.0 / (n * (n - 1.0) * p * p);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* test functions (Section 4.5 reading: phi_r = P_{r+1} - P_{r-1})             */
/* ------------------------------------------------------------------------- */
void orc_test_fn(int r, double t, double *phi, double *dphi)
{
    *phi = orc_legendre(r + 1, t) - orc_legendre(r - 1, t);
    *dphi = orc_legendre_deriv(r + 1, t) - orc_legendre_deriv(r - 1, t);
}

/* ------------------------------------------------------------------------- */
/* bilinear map of Appendix A.1                                               */
/* verts = x0,y0,x1,y1,x2,y2,x3,y3 counter-clockwise, matched to the reference */
/* corners b0(-1,-1), b1(1,-1), b2(1,1), b3(-1,1).                             */
/* ------------------------------------------------------------------------- */
static void coeffs(const double *v, double xc[4], double yc[4])
{
    const double x0 = v[0], y0 = v[1], x1 = v[2], y1 = v[3];
    const double x2 = v[4], y2 = v[5], x3 = v[6], y3 = v[7];
    xc[0] = (x0 + x1 + x2 + x3) / 4.0;
    xc[1] = (-x0 + x1 + x2 - x3) / 4.0;
    xc[2] = (-x0 - x1 + x2 + x3) / 4.0;
    xc[3] = (x0 - x1 + x2 - x3) / 4.0;
    yc[0] = (y0 + y1 + y2 + y3) / 4.0;
    yc[1] = (-y0 + y1 + y2 - y3) / 4.0;
    yc[2] = (-y0 - y1 + y2 + y3) / 4.0;
    yc[3] = (y0 - y1 + y2 - y3) / 4.0;
}

void orc_map_point(const double *verts, double xi, double eta, double *x, double *y)
{
    double xc[4], yc[4];
    coeffs(verts, xc, yc);
    *x = xc[0] + xc[1] * xi + xc[2] * eta + xc[3] * xi * eta;
    *y = yc[0] + yc[1] * xi + yc[2] * eta + yc[3] * xi * eta;
}

/* J = [[dx/dxi, dy/dxi], [dx/deta, dy/deta]] as printed in Appendix A.1 (it maps
 * (u_x, u_y) to (u_xi, u_eta)); Jinv is its true inverse; D = det J. */
void orc_jacobian(const double *verts, double xi, double eta, double J[4], double Jinv[4], double *D)
{
    double xc[4], yc[4];
    coeffs(verts, xc, yc);
    J[0] = xc[1] + xc[3] * eta;
    J[1] = yc[1] + yc[3] * eta;
    J[2] = xc[2] + xc[3] * xi;
    J[3] = yc[2] + yc[3] * xi;
    double det = J[0] * J[3] - J[1] * J[2];
    *D = det;
    Jinv[0] = J[3] / det;
    Jinv[1] = -J[1] / det;
    Jinv[2] = -J[2] / det;
    Jinv[3] = J[0] / det;
}

/* ------------------------------------------------------------------------- */
/* assembly of G_x, G_y, F and the physical quadrature points                */
/* (Section 4.4: per element, w_q * det J * physical test gradient, stacked   */
/* into [N_elem][N_test][N_quad]; Appendix A.2: F[e][k] += det J w f v).      */
/* ------------------------------------------------------------------------- */
typedef double (*orc_fn2)(double x, double y, void *user);

static double forcing(int kind, const double *par, orc_fn2 fn, void *user, double x, double y)
{
    if (kind == 1) return par[0] * sin(par[1] * x) * sin(par[2] * y);
    return fn(x, y, user);
}

/* G_x, G_y: w_q det J (grad v_k)(x_q); F: sum_q w_q det J f v_k; X: the points;
 * M (optional): w_q det J v_k(x_q), the weights of the convection term
 * int_K (b . grad u) v_k dx of the convection-diffusion weak form (Sec. 2.1). */
int orc_assemble(int64_t n_nodes, const double *xy, int64_t n_elem, const int32_t *quad,
                 int n, int nt, int f_kind, const double *f_par, orc_fn2 f_fn, void *f_user,
                 double *Gx, double *Gy, double *F, double *X, double *M, int64_t *bad_elem)
{
    if (n < 2 || nt < 1 || n_elem < 0 || !xy || !quad) return ORC_E_ARG;
    if (f_kind == 0 && !f_fn) return ORC_E_ARG;
    const int nq = n * n, ntest = nt * nt;
    double *gx = malloc(sizeof(double) * n), *gw = malloc(sizeof(double) * n);
    int status = orc_gll(n, gx, gw);
    for (int64_t e = 0; e < n_elem && status == ORC_OK; ++e) {
        double v[8];
        for (int c = 0; c < 4; ++c) {
            int32_t id = quad[e * 4 + c];
            if (id < 0 || id >= n_nodes) { status = ORC_E_MESH; break; }
            v[2 * c] = xy[2 * (int64_t)id];
            v[2 * c + 1] = xy[2 * (int64_t)id + 1];
        }
        if (status != ORC_OK) { if (bad_elem) *bad_elem = e; break; }
        for (int k = 0; k < ntest; ++k) F[e * ntest + k] = 0.0;
        for (int j = 0; j < n && status == ORC_OK; ++j) {
            for (int i = 0; i < n; ++i) {
                const int q = j * n + i;
                const double xi = gx[i], eta = gx[j], wq = gw[i] * gw[j];
                double J[4], Ji[4], D, x, y;
                orc_jacobian(v, xi, eta, J, Ji, &D);
                if (!(D > 0.0)) { status = ORC_E_MESH; if (bad_elem) *bad_elem = e; break; }
                orc_map_point(v, xi, eta, &x, &y);
                X[(e * nq + q) * 2] = x;
                X[(e * nq + q) * 2 + 1] = y;
                const double f = forcing(f_kind, f_par, f_fn, f_user, x, y);
                if (!isfinite(f)) { status = ORC_E_NONFINITE; if (bad_elem) *bad_elem = e; break; }
                for (int s = 1; s <= nt; ++s) {
                    for (int r = 1; r <= nt; ++r) {
                        const int k = (s - 1) * nt + (r - 1);
                        double pr, dpr, ps, dps;
                        orc_test_fn(r, xi, &pr, &dpr);
                        orc_test_fn(s, eta, &ps, &dps);
                        const double val = pr * ps;
                        const double dxi = dpr * ps, deta = pr * dps;
                        /* physical gradient: (v_x, v_y) = J^{-1} (v_xi, v_eta) */
                        const double vx = Ji[0] * dxi + Ji[1] * deta;
                        const double vy = Ji[2] * dxi + Ji[3] * deta;
                        const int64_t o = (e * ntest + k) * nq + q;
                        Gx[o] = wq * D * vx;
                        Gy[o] = wq * D * vy;
                        if (M) M[o] = wq * D * val;
                        F[e * ntest + k] += wq * D * f * val;
                    }
                }
            }
        }
    }
    free(gx);
    free(gw);
    return status;
}

/* ------------------------------------------------------------------------- */
/* the network of Section 2.2: u = l(T^L(...T^1(x))), T^l(a) = tanh(W_l a+b_l) */
/* flat layout: W1[H][2], b1[H], (W_l[H][H], b_l[H]) for l = 2..L,            */
/* W_out[heads][H], b_out[heads]; heads = 2 adds a second linear output, the   */
/* space-dependent diffusion coefficient eps(x, y) of Sec. 4.7.2.             */
/* Layer l is written uniformly with input width d_{l-1} (d_0 = 2, else H).   */
/* ------------------------------------------------------------------------- */
int64_t orc_n_params(int H, int L)
{
    return (int64_t)H * 2 + H + (int64_t)(L - 1) * (H * H + H) + H + 1;
}

int64_t orc_n_params_heads(int H, int L, int heads)
{
    return orc_n_params(H, L) + (int64_t)(heads - 1) * (H + 1);
}

static int64_t w_off(int H, int l) /* offset of W_l, l = 1..L+1 (L+1 is the output layer) */
{
    if (l == 1) return 0;
    return (int64_t)3 * H + (int64_t)(l - 2) * (H * H + H);
}

/* per-point forward values and tangents; arrays are [L+1][H] with row 0 the input */
typedef struct {
    int H, L, heads;
    double *a, *tx, *ty, *px, *py;
    double u, ux, uy;
    double e; /* second output (heads = 2) */
} tape;

static void tape_init(tape *t, int H, int L, int heads)
{
    t->H = H;
    t->L = L;
    t->heads = heads;
    size_t sz = sizeof(double) * (size_t)(L + 1) * (H > 2 ? H : 2);
    t->a = calloc(1, sz); t->tx = calloc(1, sz); t->ty = calloc(1, sz);
    t->px = calloc(1, sz); t->py = calloc(1, sz);
}

static void tape_free(tape *t)
{
    free(t->a); free(t->tx); free(t->ty); free(t->px); free(t->py);
}

#define ROW(arr, l) ((arr) + (size_t)(l) * stride)

/* values and the two spatial tangents (d/dx, d/dy) pushed forward layer by layer */
static void mlp_forward(const double *theta, double x, double y, tape *t)
{
    const int H = t->H, L = t->L;
    const size_t stride = (size_t)(H > 2 ? H : 2);
    double *a0 = ROW(t->a, 0), *tx0 = ROW(t->tx, 0), *ty0 = ROW(t->ty, 0);
    a0[0] = x; a0[1] = y;
    tx0[0] = 1.0; tx0[1] = 0.0;
    ty0[0] = 0.0; ty0[1] = 1.0;
    for (int l = 1; l <= L; ++l) {
        const int din = (l == 1) ? 2 : H;
        const double *W = theta + w_off(H, l);
        const double *b = W + (size_t)H * din;
        const double *ai = ROW(t->a, l - 1), *txi = ROW(t->tx, l - 1), *tyi = ROW(t->ty, l - 1);
        double *ao = ROW(t->a, l), *txo = ROW(t->tx, l), *tyo = ROW(t->ty, l);
        double *pxo = ROW(t->px, l), *pyo = ROW(t->py, l);
        for (int o = 0; o < H; ++o) {
            double z = b[o], px = 0.0, py = 0.0;
            for (int i = 0; i < din; ++i) {
                z += W[o * din + i] * ai[i];
                px += W[o * din + i] * txi[i];
                py += W[o * din + i] * tyi[i];
            }
            const double av = tanh(z);
            const double s = 1.0 - av * av; /* tanh' */
            ao[o] = av;
            pxo[o] = px;
            pyo[o] = py;
            txo[o] = s * px;
            tyo[o] = s * py;
        }
    }
    const double *Wo = theta + w_off(H, L + 1);
    const double *bo = Wo + (size_t)t->heads * H;
    const double *aL = ROW(t->a, L), *txL = ROW(t->tx, L), *tyL = ROW(t->ty, L);
    double u = bo[0], ux = 0.0, uy = 0.0;
    for (int i = 0; i < H; ++i) {
        u += Wo[i] * aL[i];
        ux += Wo[i] * txL[i];
        uy += Wo[i] * tyL[i];
    }
    t->u = u; t->ux = ux; t->uy = uy;
    t->e = 0.0;
    if (t->heads == 2) {
        double e = bo[1];
        for (int i = 0; i < H; ++i) e += Wo[H + i] * aL[i];
        t->e = e;
    }
}

/* reverse sweep: given dL/du, dL/du_x, dL/du_y (and dL/de of the second output)
 * at the point, add dL/dtheta */
static void mlp_backward(const double *theta, const tape *t, double ub, double uxb, double uyb, double eb,
                         double *grad, double *work)
{
    const int H = t->H, L = t->L;
    const size_t stride = (size_t)(H > 2 ? H : 2);
    double *abar = work, *txbar = work + H, *tybar = work + 2 * H;
    double *nabar = work + 3 * H, *ntxbar = work + 4 * H, *ntybar = work + 5 * H;
    double *zbar = work + 6 * H, *pxbar = work + 7 * H, *pybar = work + 8 * H;

    const double *Wo = theta + w_off(H, L + 1);
    double *gWo = grad + w_off(H, L + 1);
    const double *aL = ROW(t->a, L), *txL = ROW(t->tx, L), *tyL = ROW(t->ty, L);
    for (int i = 0; i < H; ++i) {
        gWo[i] += ub * aL[i] + uxb * txL[i] + uyb * tyL[i];
        abar[i] = ub * Wo[i];
        txbar[i] = uxb * Wo[i];
        tybar[i] = uyb * Wo[i];
    }
    gWo[(size_t)t->heads * H] += ub;
    if (t->heads == 2) {
        for (int i = 0; i < H; ++i) {
            gWo[H + i] += eb * aL[i];
            abar[i] += eb * Wo[H + i];
        }
        gWo[2 * (size_t)H + 1] += eb;
    }

    for (int l = L; l >= 1; --l) {
        const int din = (l == 1) ? 2 : H;
        const double *W = theta + w_off(H, l);
        double *gW = grad + w_off(H, l);
        double *gb = gW + (size_t)H * din;
        const double *ao = ROW(t->a, l), *pxo = ROW(t->px, l), *pyo = ROW(t->py, l);
        const double *ai = ROW(t->a, l - 1), *txi = ROW(t->tx, l - 1), *tyi = ROW(t->ty, l - 1);
        for (int o = 0; o < H; ++o) {
            const double s = 1.0 - ao[o] * ao[o];
            /* t = s * p  =>  p_bar = s t_bar,  s_bar = t_bar . p */
            pxbar[o] = s * txbar[o];
            pybar[o] = s * tybar[o];
            const double sbar = txbar[o] * pxo[o] + tybar[o] * pyo[o];
            /* s = 1 - a^2  =>  a_bar += -2 a s_bar;  a = tanh(z)  =>  z_bar = s a_bar */
            const double atot = abar[o] - 2.0 * ao[o] * sbar;
            zbar[o] = s * atot;
        }
        for (int o = 0; o < H; ++o) {
            for (int i = 0; i < din; ++i)
                gW[o * din + i] += zbar[o] * ai[i] + pxbar[o] * txi[i] + pybar[o] * tyi[i];
            gb[o] += zbar[o];
        }
        if (l > 1) {
            for (int i = 0; i < din; ++i) {
                double sa = 0.0, sx = 0.0, sy = 0.0;
                for (int o = 0; o < H; ++o) {
                    sa += W[o * din + i] * zbar[o];
                    sx += W[o * din + i] * pxbar[o];
                    sy += W[o * din + i] * pybar[o];
                }
                nabar[i] = sa; ntxbar[i] = sx; ntybar[i] = sy;
            }
            memcpy(abar, nabar, sizeof(double) * H);
            memcpy(txbar, ntxbar, sizeof(double) * H);
            memcpy(tybar, ntybar, sizeof(double) * H);
        }
    }
}

/* u, u_x, u_y (and the second output e) of the network at n points (for the pins) */
void orc_mlp_eval(int H, int L, int heads, const double *theta, int64_t npts, const double *xy,
                  double *u, double *ux, double *uy, double *e)
{
    tape t;
    tape_init(&t, H, L, heads);
    for (int64_t p = 0; p < npts; ++p) {
        mlp_forward(theta, xy[2 * p], xy[2 * p + 1], &t);
        if (u) u[p] = t.u;
        if (ux) ux[p] = t.ux;
        if (uy) uy[p] = t.uy;
        if (e) e[p] = t.e;
    }
    tape_free(&t);
}

/* dL/dtheta of L = sum_p (ub[p] u + uxb[p] u_x + uyb[p] u_y + eb[p] e) (for adjoint pins) */
void orc_mlp_vjp(int H, int L, int heads, const double *theta, int64_t npts, const double *xy,
                 const double *ub, const double *uxb, const double *uyb, const double *eb, double *grad)
{
    tape t;
    tape_init(&t, H, L, heads);
    double *work = malloc(sizeof(double) * 9 * (size_t)H);
    memset(grad, 0, sizeof(double) * (size_t)orc_n_params_heads(H, L, heads));
    for (int64_t p = 0; p < npts; ++p) {
        mlp_forward(theta, xy[2 * p], xy[2 * p + 1], &t);
        mlp_backward(theta, &t, ub ? ub[p] : 0.0, uxb ? uxb[p] : 0.0, uyb ? uyb[p] : 0.0, eb ? eb[p] : 0.0, grad,
                     work);
    }
    free(work);
    tape_free(&t);
}

/* ------------------------------------------------------------------------- */
/* residual from given solution gradients at the quadrature points            */
/* R[e,k] = eps * sum_q (u_x G_x + u_y G_y)[e,k,q]                            */
/*        + sum_q (b_x u_x + b_y u_y) M[e,k,q] - F[e,k]                       */
/* (Algorithm 3; the convection term of the convection-diffusion weak form,   */
/* Sec. 2.1, when M is given).  With epsq (per point) the diffusion          */
/* coefficient varies in space (Sec. 4.7.2): eps * (...) becomes             */
/* sum_q epsq[q] (u_x G_x + u_y G_y)[q].                                      */
/* ------------------------------------------------------------------------- */
void orc_residual(int64_t n_elem, int nq, int ntest, const double *Gx, const double *Gy,
                  const double *F, const double *ux, const double *uy, double eps,
                  const double *M, double cbx, double cby, const double *epsq, double *R)
{
    for (int64_t e = 0; e < n_elem; ++e) {
        for (int k = 0; k < ntest; ++k) {
            double acc = 0.0, conv = 0.0;
            for (int q = 0; q < nq; ++q) {
                const int64_t o = (e * ntest + k) * nq + q;
                const double w = epsq ? epsq[e * nq + q] : 1.0;
                acc += w * (ux[e * nq + q] * Gx[o] + uy[e * nq + q] * Gy[o]);
                if (M) conv += (cbx * ux[e * nq + q] + cby * uy[e * nq + q]) * M[o];
            }
            R[e * ntest + k] = (epsq ? 1.0 : eps) * acc + conv - F[e * ntest + k];
        }
    }
}

/* ------------------------------------------------------------------------- */
/* total loss and gradient                                                    */
/* L = c_v sum_{e,k} R^2 + tau mean_b (u_b - g_b)^2 + gamma mean_s (u_s - d_s)^2 */
/* loss[0..3] = L, L_v, L_b, L_s (L_b, L_s unweighted means)                  */
/* ------------------------------------------------------------------------- */
int orc_loss_grad(int64_t n_elem, int nq, int ntest, const double *Gx, const double *Gy,
                  const double *F, const double *X, const double *M, double cbx, double cby,
                  int64_t n_bnd, const double *bxy, const double *bg,
                  int64_t n_sen, const double *sxy, const double *su,
                  int H, int L, int heads, const double *theta, double eps, double tau, double gamma,
                  double cv, double *loss, double *grad, double *grad_eps, double *R_out)
{
    /* heads = 2: the network's second output is the space-dependent diffusion
     * coefficient e(x, y) (Sec. 4.7.2); the diffusion term becomes
     * sum_q e(x_q) (u_x G_x + u_y G_y), and eps is not used */
    if (H < 1 || L < 1 || nq < 1 || ntest < 1 || heads < 1 || heads > 2) return ORC_E_ARG;
    const int64_t np_ = orc_n_params_heads(H, L, heads);
    if (grad) memset(grad, 0, sizeof(double) * (size_t)np_);
    tape *tp = malloc(sizeof(tape) * (size_t)nq);
    for (int q = 0; q < nq; ++q) tape_init(&tp[q], H, L, heads);
    double *work = malloc(sizeof(double) * 9 * (size_t)H);
    double *A = malloc(sizeof(double) * ntest), *R = malloc(sizeof(double) * ntest);
    double Lv = 0.0, geps = 0.0;

    /* variational term, one element at a time (the loop of Section 3.1) */
    for (int64_t e = 0; e < n_elem; ++e) {
        for (int q = 0; q < nq; ++q)
            mlp_forward(theta, X[(e * nq + q) * 2], X[(e * nq + q) * 2 + 1], &tp[q]);
        double le = 0.0;
        for (int k = 0; k < ntest; ++k) {
            double acc = 0.0, conv = 0.0;
            for (int q = 0; q < nq; ++q) {
                const int64_t o = (e * ntest + k) * nq + q;
                const double w = heads == 2 ? tp[q].e : 1.0;
                acc += w * (tp[q].ux * Gx[o] + tp[q].uy * Gy[o]);
                if (M) conv += (cbx * tp[q].ux + cby * tp[q].uy) * M[o];
            }
            A[k] = acc;
            R[k] = (heads == 2 ? 1.0 : eps) * acc + conv - F[e * ntest + k];
            if (R_out) R_out[e * ntest + k] = R[k];
            le += R[k] * R[k];
        }
        Lv += cv * le;
        if (!grad && !grad_eps) continue;
        /* dL/dR = 2 c_v R ; dL/deps = sum_k dL/dR A ;                         */
        /* dL/du_x[q] = sum_k dL/dR (eps G_x + b_x M)  (and y likewise), with  */
        /* eps -> e(x_q) for two outputs, and then                             */
        /* dL/de[q] = sum_k dL/dR (u_x G_x + u_y G_y)[q]                        */
        if (heads == 1)
            for (int k = 0; k < ntest; ++k) geps += 2.0 * cv * R[k] * A[k];
        if (grad) {
            for (int q = 0; q < nq; ++q) {
                const double w = heads == 2 ? tp[q].e : eps;
                double bx = 0.0, by = 0.0, be = 0.0;
                for (int k = 0; k < ntest; ++k) {
                    const int64_t o = (e * ntest + k) * nq + q;
                    bx += 2.0 * cv * R[k] * w * Gx[o];
                    by += 2.0 * cv * R[k] * w * Gy[o];
                    if (M) {
                        bx += 2.0 * cv * R[k] * cbx * M[o];
                        by += 2.0 * cv * R[k] * cby * M[o];
                    }
                    be += 2.0 * cv * R[k] * (tp[q].ux * Gx[o] + tp[q].uy * Gy[o]);
                }
                mlp_backward(theta, &tp[q], 0.0, bx, by, heads == 2 ? be : 0.0, grad, work);
            }
        }
    }

    /* Dirichlet boundary term (Section 2.2) */
    double Lb = 0.0, Ls = 0.0;
    for (int64_t b = 0; b < n_bnd; ++b) {
        mlp_forward(theta, bxy[2 * b], bxy[2 * b + 1], &tp[0]);
        const double d = tp[0].u - bg[b];
        Lb += d * d / (double)n_bnd;
        if (grad) mlp_backward(theta, &tp[0], tau * 2.0 * d / (double)n_bnd, 0.0, 0.0, 0.0, grad, work);
    }
    /* sensor data term (Section 4.7) */
    for (int64_t s = 0; s < n_sen; ++s) {
        mlp_forward(theta, sxy[2 * s], sxy[2 * s + 1], &tp[0]);
        const double d = tp[0].u - su[s];
        Ls += d * d / (double)n_sen;
        if (grad) mlp_backward(theta, &tp[0], gamma * 2.0 * d / (double)n_sen, 0.0, 0.0, 0.0, grad, work);
    }
    loss[0] = Lv + tau * Lb + gamma * Ls;
    loss[1] = Lv;
    loss[2] = Lb;
    loss[3] = Ls;
    if (grad_eps) *grad_eps = geps;

    for (int q = 0; q < nq; ++q) tape_free(&tp[q]);
    free(tp);
    free(work);
    free(A);
    free(R);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Adam (Kingma and Ba, Algorithm 1): bias-corrected first and second moments */
/* ------------------------------------------------------------------------- */
void orc_adam(int64_t n, double *theta, const double *g, double *m, double *v, int64_t t,
              double lr, double b1, double b2, double eps)
{
    const double c1 = 1.0 - pow(b1, (double)t);
    const double c2 = 1.0 - pow(b2, (double)t);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        const double mh = m[i] / c1;
        const double vh = v[i] / c2;
        theta[i] -= lr * mh / (sqrt(vh) + eps);
    }
}
