/*
 * oracle.c -- plain, slow CPU reference for the partitioned 3D Gaussian
 * splatting rasterizer of RetinaGS (arXiv 2406.11836).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the HIP library.
 *
 * What it computes, and where the paper defines it:
 *   - 3D Gaussian, opacity, SH colour and EWA projection (Sec. 3.1, Eq. 1).
 *   - Front-to-back alpha blending in depth order (Sec. 3.1, Eq. 2).
 *   - Per-subset partial colour and transmittance with the indicator of the
 *     ray's crossing point (Sec. 3.2, Eq. 3, Eq. 4, Eq. 6).
 *   - Merge of the partials in the order the ray visits the subspaces
 *     (Sec. 3.2, Eq. 5), whose equivalence with Eq. 2 is the appendix proof.
 *   - KD-tree partition by equal-count bisection and the overlapping subsets
 *     N_k with the margin D_i (Sec. 3.3).
 *   - Reverse-mode derivatives of all of the above (the manager sends the
 *     loss gradient back to every subset, Sec. 3.4) and the L1/SSIM loss.
 *
 * Two modes for the discrete decisions (which Gaussian touches which pixel,
 * in which cell, the screen rectangle, the cell set):
 *   mode 0 (mirror32): decisions follow the GPU kernels' fixed operation
 *            sequence (an fp64 covariance chain rounded once to fp32, then
 *            fp32 tests), so that integer outputs can be compared bit for
 *            bit;
 *   mode 1 (exact64):  decisions are taken in fp64.
 * Values (sigma, colour, blending, merge, gradients) are always fp64.
 * Compile with -ffp-contract=off and without -ffast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXK 64

/* ------------------------------------------------------------------ */
/* camera                                                              */
/* ------------------------------------------------------------------ */
/* Packed camera, 25 doubles:
 *   [0..8]  R, world->camera rotation, row-major (p_cam = R p + t)
 *   [9..11] t
 *   [12..14] o, camera centre in world coordinates
 *   [15] fx [16] fy [17] cx [18] cy [19] width [20] height [21] z_near
 *   [22..24] background colour
 * Pixel (x, y) is sampled at image coordinates (x + 0.5, y + 0.5); camera
 * axes are x right, y down, z forward.                                 */
typedef struct {
    double R[9], t[3], o[3], fx, fy, cx, cy, znear, bg[3];
    int W, H;
} Cam;

static void cam_unpack(const double *c, Cam *m) {
    memcpy(m->R, c, 9 * sizeof(double));
    memcpy(m->t, c + 9, 3 * sizeof(double));
    memcpy(m->o, c + 12, 3 * sizeof(double));
    m->fx = c[15]; m->fy = c[16]; m->cx = c[17]; m->cy = c[18];
    m->W = (int)c[19]; m->H = (int)c[20]; m->znear = c[21];
    m->bg[0] = c[22]; m->bg[1] = c[23]; m->bg[2] = c[24];
}

/* ------------------------------------------------------------------ */
/* real spherical harmonics                                            */
/* ------------------------------------------------------------------ */
/* Real orthonormal SH with the Condon-Shortley phase, index j = l*l+l+m.
 * Y_l^m = N_lm * P_l^(|m|)(z) * A_m(x, y), with P_l^(k) the k-th
 * derivative of the Legendre polynomial, A_m = Re (x+iy)^m for m > 0,
 * Im (x+iy)^|m| for m < 0, 1 for m = 0, and
 * N_lm = sqrt(2) (-1)^|m| K_l^|m| (m != 0), K_l^0 (m = 0),
 * K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).
 * Built from the definition, not from tabulated constants.  The value and
 * the gradient of the polynomial extension to R^3 are returned.        */
#define SH_LMAX 3
static double fact(int k) { double r = 1; for (int i = 2; i <= k; i++) r *= i; return r; }

/* Legendre polynomial coefficients: P[l][p] is the z^p coefficient. */
static void legendre_coeffs(double P[SH_LMAX + 1][SH_LMAX + 1]) {
    memset(P, 0, sizeof(double) * (SH_LMAX + 1) * (SH_LMAX + 1));
    P[0][0] = 1.0;
    if (SH_LMAX >= 1) P[1][1] = 1.0;
    for (int l = 1; l < SH_LMAX; l++) {
        /* (l+1) P_{l+1} = (2l+1) z P_l - l P_{l-1}  (Bonnet) */
        for (int p = 0; p <= SH_LMAX; p++) {
            double v = 0;
            if (p >= 1) v += (2 * l + 1) * P[l][p - 1];
            v -= l * P[l - 1][p];
            P[l + 1][p] = v / (l + 1);
        }
    }
}

static double poly_eval(const double *c, int deg, double z) {
    double r = 0;
    for (int p = deg; p >= 0; p--) r = r * z + c[p];
    return r;
}

/* Y[j] and dY[j][3] (gradient w.r.t. x, y, z of the polynomial form) */
void orc_sh_basis(int D, const double *dir, double *Y, double *dY) {
    double P[SH_LMAX + 1][SH_LMAX + 1];
    legendre_coeffs(P);
    double x = dir[0], y = dir[1], z = dir[2];
    /* powers of (x + i y) */
    double re[SH_LMAX + 1], im[SH_LMAX + 1];
    re[0] = 1; im[0] = 0;
    for (int k = 1; k <= SH_LMAX; k++) {
        re[k] = re[k - 1] * x - im[k - 1] * y;
        im[k] = re[k - 1] * y + im[k - 1] * x;
    }
    for (int l = 0; l <= D; l++) {
        for (int m = -l; m <= l; m++) {
            int am = m < 0 ? -m : m;
            /* am-th derivative of P_l, and its derivative */
            double d[SH_LMAX + 1] = {0}, dd[SH_LMAX + 1] = {0};
            for (int p = 0; p <= SH_LMAX; p++) d[p] = P[l][p];
            for (int k = 0; k < am; k++)
                for (int p = 0; p <= SH_LMAX; p++) d[p] = (p + 1 <= SH_LMAX) ? (p + 1) * d[p + 1] : 0;
            for (int p = 0; p <= SH_LMAX; p++) dd[p] = (p + 1 <= SH_LMAX) ? (p + 1) * d[p + 1] : 0;
            double K = sqrt((2 * l + 1) / (4 * M_PI) * fact(l - am) / fact(l + am));
            double N = (m == 0) ? K : sqrt(2.0) * ((am & 1) ? -1.0 : 1.0) * K;
            double Pz = poly_eval(d, SH_LMAX, z), dPz = poly_eval(dd, SH_LMAX, z);
            double A, Ax, Ay;
            if (m == 0) { A = 1; Ax = 0; Ay = 0; }
            else if (m > 0) { A = re[am]; Ax = am * re[am - 1]; Ay = -am * im[am - 1]; }
            else { A = im[am]; Ax = am * im[am - 1]; Ay = am * re[am - 1]; }
            int j = l * l + l + m;
            Y[j] = N * Pz * A;
            if (dY) {
                dY[3 * j + 0] = N * Pz * Ax;
                dY[3 * j + 1] = N * Pz * Ay;
                dY[3 * j + 2] = N * dPz * A;
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* KD tree (Sec. 3.3)                                                  */
/* ------------------------------------------------------------------ */
/* IEEE totalOrder key of a non-NaN float: larger key <=> larger value,
 * with -0 < +0.                                                        */
static uint32_t f2key(float f) {
    uint32_t u; memcpy(&u, &f, 4);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
static int cmp_u32(const void *a, const void *b) {
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

/* Depth-L tree over the centres; at level l the axis is l mod 3 (X, Y, Z
 * in turn) and the split value is the floor(n/2)-th smallest coordinate of
 * the node's members (0-based, IEEE total order); members with coordinate
 * < split go left, the rest right.  An empty node splits at the midpoint
 * of its finite bounds (one finite bound: that bound; none: 0).
 * Leaves are numbered by their root-to-leaf path bits (left 0, right 1),
 * most significant bit first; nodes are stored in heap order.
 * own_mask marks the paper's subsets N_k: centre inside the leaf box
 * inflated by D_i = d_factor * max_a exp(log_scale_a) on every face. */
/* rule 0: the equal-count bisection above (the paper's KD tree).
 * rule 1: the fixed-size partition the paper compares it with (Sec. 4.2,
 * Table 2): every node is cut at the midpoint of its extent, starting from
 * the bounding box of all centres, so that the leaves are the blocks of a
 * uniform grid (2^ceil(L/3) x 2^ceil((L-1)/3) x 2^floor(L/3)); split =
 * 0.5f * (lo + hi) in fp32 (0 when there are no centres).  Boxes, leaf
 * numbering, counts and N_k are as for rule 0.                          */
int orc_kd_partition(int64_t n, const double *means, const double *log_scales, int L,
                     double d_factor, int rule, float *split, uint8_t *axis, float *box_lo,
                     float *box_hi, int32_t *center_cell, int32_t *counts, uint32_t *own_mask) {
    if (L < 0 || L > 6 || rule < 0 || rule > 1) return -1;
    int K = 1 << L;
    int32_t *node = (int32_t *)calloc(n > 0 ? n : 1, sizeof(int32_t)); /* heap index */
    uint32_t *tmp = (uint32_t *)malloc(sizeof(uint32_t) * (n > 0 ? n : 1));
    /* node bounds (for empty nodes and leaf boxes) */
    float lo[2 * ORC_MAXK][3], hi[2 * ORC_MAXK][3];
    for (int a = 0; a < 3; a++) { lo[0][a] = -INFINITY; hi[0][a] = INFINITY; }
    /* grid rule: each node's extent, from the bounding box of the centres */
    float glo[2 * ORC_MAXK][3], ghi[2 * ORC_MAXK][3];
    for (int a = 0; a < 3; a++) {
        glo[0][a] = INFINITY; ghi[0][a] = -INFINITY;
        for (int64_t i = 0; i < n; i++) {
            float c = (float)means[a * n + i];
            if (c < glo[0][a]) glo[0][a] = c;
            if (c > ghi[0][a]) ghi[0][a] = c;
        }
    }
    for (int l = 0; l < L; l++) {
        int a = l % 3;
        int first = (1 << l) - 1, cnt = 1 << l;
        for (int nd = first; nd < first + cnt; nd++) {
            int64_t m = 0;
            for (int64_t i = 0; i < n; i++)
                if (node[i] == nd) tmp[m++] = f2key((float)means[a * n + i]);
            float s;
            if (rule == 1) {
                s = (isfinite(glo[nd][a]) && isfinite(ghi[nd][a])) ? 0.5f * (glo[nd][a] + ghi[nd][a]) : 0.0f;
                for (int b = 0; b < 3; b++) {
                    glo[2 * nd + 1][b] = glo[nd][b]; ghi[2 * nd + 1][b] = ghi[nd][b];
                    glo[2 * nd + 2][b] = glo[nd][b]; ghi[2 * nd + 2][b] = ghi[nd][b];
                }
                ghi[2 * nd + 1][a] = s;
                glo[2 * nd + 2][a] = s;
            } else if (m == 0) {
                float blo = lo[nd][a], bhi = hi[nd][a];
                if (isfinite(blo) && isfinite(bhi)) s = 0.5f * (blo + bhi);
                else if (isfinite(blo)) s = blo;
                else if (isfinite(bhi)) s = bhi;
                else s = 0.0f;
            } else {
                qsort(tmp, (size_t)m, sizeof(uint32_t), cmp_u32);
                uint32_t k = tmp[m / 2];
                uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
                memcpy(&s, &u, 4);
            }
            split[nd] = s;
            axis[nd] = (uint8_t)a;
            for (int b = 0; b < 3; b++) {
                lo[2 * nd + 1][b] = lo[nd][b]; hi[2 * nd + 1][b] = hi[nd][b];
                lo[2 * nd + 2][b] = lo[nd][b]; hi[2 * nd + 2][b] = hi[nd][b];
            }
            hi[2 * nd + 1][a] = s;
            lo[2 * nd + 2][a] = s;
        }
        for (int64_t i = 0; i < n; i++) {
            int nd = node[i];
            float c = (float)means[a * n + i];
            node[i] = (c < split[nd]) ? 2 * nd + 1 : 2 * nd + 2;
        }
    }
    for (int k = 0; k < K; k++) {
        counts[k] = 0;
        for (int a = 0; a < 3; a++) {
            box_lo[a * K + k] = lo[K - 1 + k][a];
            box_hi[a * K + k] = hi[K - 1 + k][a];
        }
    }
    int W = (K + 31) / 32;
    for (int64_t i = 0; i < n; i++) {
        int leaf = node[i] - (K - 1);
        center_cell[i] = leaf;
        counts[leaf]++;
        float s0 = (float)exp((double)(float)log_scales[0 * n + i]);
        float s1 = (float)exp((double)(float)log_scales[1 * n + i]);
        float s2 = (float)exp((double)(float)log_scales[2 * n + i]);
        float Di = (float)d_factor * fmaxf(fmaxf(s0, s1), s2);
        for (int w = 0; w < W; w++) own_mask[i * W + w] = 0;
        for (int k = 0; k < K; k++) {
            int in = 1;
            for (int a = 0; a < 3; a++) {
                float u = (float)means[a * n + i];
                /* outward normal -e_a, offset lo: lo - u <= D; normal +e_a: u - hi <= D */
                if (!((box_lo[a * K + k] - u) <= Di)) in = 0;
                if (!((u - box_hi[a * K + k]) <= Di)) in = 0;
            }
            if (in) own_mask[i * W + k / 32] |= 1u << (k % 32);
        }
    }
    free(node); free(tmp);
    return 0;
}

/* Per-view order of the cells along any ray from o (Eq. 5's o_l): in-order
 * traversal, near child first; the near child is the left one iff
 * o_axis < split (a centre on the plane lies in the right, half-open box). */
static void order_rec(int nd, int depth, int L, const float *split, const double *o,
                      int32_t *order, int *pos) {
    int K = 1 << L;
    if (depth == L) { order[(*pos)++] = nd - (K - 1); return; }
    int a = depth % 3;
    int left_first = ((float)o[a] < split[nd]);
    if (left_first) {
        order_rec(2 * nd + 1, depth + 1, L, split, o, order, pos);
        order_rec(2 * nd + 2, depth + 1, L, split, o, order, pos);
    } else {
        order_rec(2 * nd + 2, depth + 1, L, split, o, order, pos);
        order_rec(2 * nd + 1, depth + 1, L, split, o, order, pos);
    }
}
void orc_cell_order(int L, const float *split, const double *o, int32_t *order, int32_t *rank_of) {
    int pos = 0;
    order_rec(0, 0, L, split, o, order, &pos);
    for (int r = 0; r < (1 << L); r++) rank_of[order[r]] = r;
}

/* ------------------------------------------------------------------ */
/* projection (Sec. 3.1)                                               */
/* ------------------------------------------------------------------ */
/* Output per Gaussian:
 *   dec32[10] fp32 decision quantities: mx, my, ca, cb, cc, tau, z, alpha, k, e
 *             (d^2 = ca (dx + k dy)^2 + e dy^2; cb, cc for reference)
 *   val[12]   fp64 values: mx, my, ca, cb, cc, alpha, z, r, g, b, tau, det
 *   rect[4]   pixel rectangle x_lo, x_hi, y_lo, y_hi (decision mode)
 *   vis       1 if the Gaussian survives culling (decision mode)
 *   cellmask  KD leaves the footprint can touch (decision mode)
 *   count     |cellmask| * tiles (16 px) in the row spans of row_span32
 *             (decision mode; exact64 mode: every tile of the rectangle)
 * Conic (ca, cb, cc) is the inverse of the screen covariance:
 * d^2 = ca dx^2 + 2 cb dx dy + cc dy^2.                                 */

typedef struct { double mx, my, ca, cb, cc, alpha, z, rgb[3], tau, det; int vis; } P64;

/* fp64 projection of Gaussian i (the value path, and the decision path in
 * exact64 mode).  Culling: zero quaternion, z <= z_near, det <= 0,
 * alpha < 1/255 (tau < 0).  The rectangle test is done by the caller.   */
static void proj64(int64_t n, int D, const double *means, const double *ls, const double *q,
                   const double *op, const double *sh, const Cam *c, int64_t i, P64 *p) {
    memset(p, 0, sizeof(*p));
    double mu[3] = {means[i], means[n + i], means[2 * n + i]};
    double s[3] = {exp(ls[i]), exp(ls[n + i]), exp(ls[2 * n + i])};
    double alpha = 1.0 / (1.0 + exp(-op[i]));
    double qw = q[i], qx = q[n + i], qy = q[2 * n + i], qz = q[3 * n + i];
    double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    if (!(qn > 0)) return;
    double w = qw / qn, x = qx / qn, y = qy / qn, z = qz / qn;
    double Rq[3][3] = {
        {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
        {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
        {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
    double M[3][3], S[3][3];
    for (int a = 0; a < 3; a++) for (int b = 0; b < 3; b++) M[a][b] = Rq[a][b] * s[b];
    for (int a = 0; a < 3; a++) for (int b = 0; b < 3; b++)
        S[a][b] = M[a][0] * M[b][0] + M[a][1] * M[b][1] + M[a][2] * M[b][2];
    double t[3];
    for (int a = 0; a < 3; a++)
        t[a] = c->R[3 * a] * mu[0] + c->R[3 * a + 1] * mu[1] + c->R[3 * a + 2] * mu[2] + c->t[a];
    double zc = t[2];
    if (!(zc > c->znear)) return;
    double gx = 1.3 * (fmax(c->cx, c->W - c->cx) / c->fx);
    double gy = 1.3 * (fmax(c->cy, c->H - c->cy) / c->fy);
    double xz = t[0] / zc, yz = t[1] / zc;
    double xg = fmin(fmax(xz, -gx), gx) * zc, yg = fmin(fmax(yz, -gy), gy) * zc;
    double J[2][3] = {{c->fx / zc, 0, -c->fx * xg / (zc * zc)}, {0, c->fy / zc, -c->fy * yg / (zc * zc)}};
    double T[2][3], U[2][3];
    for (int a = 0; a < 2; a++) for (int b = 0; b < 3; b++)
        T[a][b] = J[a][0] * c->R[b] + J[a][1] * c->R[3 + b] + J[a][2] * c->R[6 + b];
    for (int a = 0; a < 2; a++) for (int b = 0; b < 3; b++)
        U[a][b] = T[a][0] * S[0][b] + T[a][1] * S[1][b] + T[a][2] * S[2][b];
    double s00 = U[0][0] * T[0][0] + U[0][1] * T[0][1] + U[0][2] * T[0][2] + 0.3;
    double s01 = U[0][0] * T[1][0] + U[0][1] * T[1][1] + U[0][2] * T[1][2];
    double s11 = U[1][0] * T[1][0] + U[1][1] * T[1][1] + U[1][2] * T[1][2] + 0.3;
    double det = s00 * s11 - s01 * s01;
    if (!(det > 0)) return;
    p->ca = s11 / det; p->cb = -s01 / det; p->cc = s00 / det; p->det = det;
    p->mx = c->fx * xz + c->cx; p->my = c->fy * yz + c->cy;
    p->alpha = alpha; p->z = zc;
    p->tau = fmin(9.0, 2.0 * log(255.0 * alpha));
    if (!(p->tau >= 0)) return;
    if (!(isfinite(p->mx) && isfinite(p->my))) return;
    /* colour: 0.5 + sum_j f_j Y_j(dir), clamped at 0; dir from the camera centre */
    double d[3] = {mu[0] - c->o[0], mu[1] - c->o[1], mu[2] - c->o[2]};
    double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    d[0] /= dn; d[1] /= dn; d[2] /= dn;
    double Y[16];
    orc_sh_basis(D, d, Y, NULL);
    int nc = (D + 1) * (D + 1);
    for (int ch = 0; ch < 3; ch++) {
        double v = 0.5;
        for (int j = 0; j < nc; j++) v += sh[(3 * j + ch) * n + i] * Y[j];
        p->rgb[ch] = v > 0 ? v : 0;
    }
    p->vis = 1;
}

/* fp32 decision path with a fixed operation order (mirror32).  Every
 * step below is one IEEE binary32 operation; transcendentals are taken in
 * fp64 and rounded once to fp32.                                       */
typedef struct { float mx, my, ca, cb, cc, tau, z, alpha, k, e, rk; int vis; float s00, s11; } P32;

/* Decision-mode projection.  Inputs are the fp32 parameters and camera;
 * the scale and opacity activations are fp64 transcendentals rounded once
 * to fp32.  Everything from the quaternion to the inverse of the screen
 * covariance runs in fp64 (+, -, *, /, sqrt only: IEEE correctly rounded,
 * so any machine gets the same bits) and is rounded once to fp32: the
 * inverse of a nearly singular covariance (a needle-like footprint) keeps
 * its accuracy, which an fp32 product chain does not.  The quadratic form
 * is kept in a factored, cancellation-free shape,
 *     d^2 = ca u^2 + e dy^2,  u = dx + k dy,
 * with ca = s11/det, k = -s01/s11 and e = 1/s11 (ca cc - cb^2 = ca e);
 * cb and cc are also returned for reference.  rk = sqrt(1 + k^2 ca/e) =
 * sqrt(s00 s11 / det) measures the elongation.                          */
static void proj32(int64_t n, const double *means, const double *ls, const double *q,
                   const double *op, const Cam *c, int64_t i, P32 *p) {
    memset(p, 0, sizeof(*p));
    double mu0 = (float)means[i], mu1 = (float)means[n + i], mu2 = (float)means[2 * n + i];
    float s0 = (float)exp((double)(float)ls[i]);
    float s1 = (float)exp((double)(float)ls[n + i]);
    float s2 = (float)exp((double)(float)ls[2 * n + i]);
    float alpha = (float)(1.0 / (1.0 + exp(-(double)(float)op[i])));
    double qw = (float)q[i], qx = (float)q[n + i], qy = (float)q[2 * n + i], qz = (float)q[3 * n + i];
    double qq = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
    if (!(qq > 0.0)) return;
    double qn = sqrt(qq);
    double w = qw / qn, x = qx / qn, y = qy / qn, z = qz / qn;
    double r[3][3];
    r[0][0] = 1.0 - 2.0 * (y * y + z * z);
    r[0][1] = 2.0 * (x * y - w * z);
    r[0][2] = 2.0 * (x * z + w * y);
    r[1][0] = 2.0 * (x * y + w * z);
    r[1][1] = 1.0 - 2.0 * (x * x + z * z);
    r[1][2] = 2.0 * (y * z - w * x);
    r[2][0] = 2.0 * (x * z - w * y);
    r[2][1] = 2.0 * (y * z + w * x);
    r[2][2] = 1.0 - 2.0 * (x * x + y * y);
    double sc[3] = {s0, s1, s2};
    double M[3][3], S[3][3];
    for (int a = 0; a < 3; a++) for (int b = 0; b < 3; b++) M[a][b] = r[a][b] * sc[b];
    for (int a = 0; a < 3; a++) for (int b = 0; b < 3; b++)
        S[a][b] = (M[a][0] * M[b][0] + M[a][1] * M[b][1]) + M[a][2] * M[b][2];
    double R[9];
    for (int k = 0; k < 9; k++) R[k] = (float)c->R[k];
    double tc[3];
    for (int a = 0; a < 3; a++)
        tc[a] = ((R[3 * a] * mu0 + R[3 * a + 1] * mu1) + R[3 * a + 2] * mu2) + (double)(float)c->t[a];
    double zc = tc[2];
    if (!(zc > (double)(float)c->znear)) return;
    float fx32 = (float)c->fx, fy32 = (float)c->fy, cx32 = (float)c->cx, cy32 = (float)c->cy;
    float Wf = (float)c->W, Hf = (float)c->H;
    double gx = 1.3f * (fmaxf(cx32, Wf - cx32) / fx32);
    double gy = 1.3f * (fmaxf(cy32, Hf - cy32) / fy32);
    double fx = fx32, fy = fy32, cx = cx32, cy = cy32;
    double xz = tc[0] / zc, yz = tc[1] / zc;
    double xg = fmin(fmax(xz, -gx), gx) * zc;
    double yg = fmin(fmax(yz, -gy), gy) * zc;
    double zz = zc * zc;
    double J00 = fx / zc, J02 = -(fx * xg) / zz, J11 = fy / zc, J12 = -(fy * yg) / zz;
    double T[2][3], U[2][3];
    for (int b = 0; b < 3; b++) {
        T[0][b] = J00 * R[b] + J02 * R[6 + b];
        T[1][b] = J11 * R[3 + b] + J12 * R[6 + b];
    }
    for (int a = 0; a < 2; a++) for (int b = 0; b < 3; b++)
        U[a][b] = (T[a][0] * S[0][b] + T[a][1] * S[1][b]) + T[a][2] * S[2][b];
    double s00 = ((U[0][0] * T[0][0] + U[0][1] * T[0][1]) + U[0][2] * T[0][2]) + 0.3;
    double s01 = (U[0][0] * T[1][0] + U[0][1] * T[1][1]) + U[0][2] * T[1][2];
    double s11 = ((U[1][0] * T[1][0] + U[1][1] * T[1][1]) + U[1][2] * T[1][2]) + 0.3;
    double det = s00 * s11 - s01 * s01;
    if (!(det > 0.0)) return;
    p->ca = (float)(s11 / det); p->cb = (float)(-s01 / det); p->cc = (float)(s00 / det);
    p->k = (float)(-s01 / s11); p->e = (float)(1.0 / s11);
    p->rk = sqrtf(1.0f + (p->k * p->k) * (p->ca / p->e));
    p->mx = (float)(fx * xz + cx); p->my = (float)(fy * yz + cy);
    p->z = (float)zc; p->alpha = alpha; p->s00 = (float)s00; p->s11 = (float)s11;
    float tau = fminf(9.0f, (float)(2.0 * log(255.0 * (double)alpha)));
    p->tau = tau;
    if (!(tau >= 0.0f)) return;
    if (!(isfinite(p->mx) && isfinite(p->my))) return;
    p->vis = 1;
}

/* Screen rectangle of sample pixels that can satisfy d^2 <= tau: the
 * ellipse's x-extent is sqrt(tau * s00) (min over dy of d^2 is
 * dx^2 / s00).  Padding: 1e-3 px, a relative 1e-5, and a relative
 * 2^-20 rk.  The per-pixel test in fp32 evaluates u = dx + k dy with an
 * absolute error up to about 2^-24 |dx|, which moves ca u^2 near the edge
 * by up to about 2^-23 tau rk (ca s00 = rk^2); the ellipse of the rounded
 * (ca, k, e) is within a few 2^-24 of the exact one.
 * Returns 0 when the rectangle is empty.                                */
static int rect32(const P32 *p, const Cam *c, int rect[4]) {
    float pad = 1.00001f + 0x1p-20f * p->rk;
    float ex = sqrtf(p->tau * p->s00) * pad + 1e-3f;
    float ey = sqrtf(p->tau * p->s11) * pad + 1e-3f;
    float xlo = fmaxf(ceilf((p->mx - ex) - 0.5f), 0.0f);
    float xhi = fminf(floorf((p->mx + ex) - 0.5f), (float)(c->W - 1));
    float ylo = fmaxf(ceilf((p->my - ey) - 0.5f), 0.0f);
    float yhi = fminf(floorf((p->my + ey) - 0.5f), (float)(c->H - 1));
    if (!(xlo <= xhi) || !(ylo <= yhi)) return 0;
    rect[0] = (int)xlo; rect[1] = (int)xhi; rect[2] = (int)ylo; rect[3] = (int)yhi;
    return 1;
}
static int rect64(const P64 *p, const Cam *c, int rect[4]) {
    double s00 = p->cc * p->det, s11 = p->ca * p->det;
    double ex = sqrt(p->tau * s00) * 1.00001 + 1e-3;
    double ey = sqrt(p->tau * s11) * 1.00001 + 1e-3;
    double xlo = fmax(ceil(p->mx - ex - 0.5), 0.0), xhi = fmin(floor(p->mx + ex - 0.5), c->W - 1.0);
    double ylo = fmax(ceil(p->my - ey - 0.5), 0.0), yhi = fmin(floor(p->my + ey - 0.5), c->H - 1.0);
    if (!(xlo <= xhi) || !(ylo <= yhi)) return 0;
    rect[0] = (int)xlo; rect[1] = (int)xhi; rect[2] = (int)ylo; rect[3] = (int)yhi;
    return 1;
}

/* Tile columns [*c0, *c1] of tile row ty (16 px rows) that hold a pixel
 * centre of the rectangle able to satisfy d^2 <= tau; *c0 > *c1 when none.
 * Decision mode only: fp32, fixed order, no contraction; d is a dec32 row.
 *
 * In the factored form d^2 = ca u^2 + e dy^2, u = dx + k dy, the chord of
 * {d^2 <= tau} at height dy is dx = -k dy +- sqrt((tau - e dy^2) / ca).
 * Its right end is concave in dy and largest at the height of the
 * ellipse's rightmost point, dy_r = -k sqrt(ca tau / (e (e + k^2 ca)));
 * its left end is convex and smallest at -dy_r.  Over the row's band of
 * pixel-centre heights [ly, hy] the x-extent is therefore the chord ends
 * at clamp(dy_r) and clamp(-dy_r).  tau is enlarged to tau (1 + 2^-18
 * (1 + rk)), above what rounding of the per-pixel test can accept (see
 * rect32), and the ends are padded by 1/64 px plus 2^-16 of their size.
 * Every term is a sum of non-negative parts: no cancellation for any
 * elongation.  A non-finite end keeps the rectangle's bound.            */
static void row_span32(const float *d, const int r[4], int ty, int *c0, int *c1) {
    float mx = d[0], my = d[1], ca = d[2], tau = d[5], k = d[8], e = d[9];
    float rk = sqrtf(1.0f + (k * k) * (ca / e));
    float taup = tau + tau * (0x1p-18f * (1.0f + rk));
    float dyr = -(k * sqrtf((ca * taup) / (e * (e + (k * k) * ca))));
    int y0 = ty * 16 > r[2] ? ty * 16 : r[2];
    int y1 = ty * 16 + 15 < r[3] ? ty * 16 + 15 : r[3];
    float ly = ((float)y0 + 0.5f) - my, hy = ((float)y1 + 0.5f) - my;
    float dR = fminf(fmaxf(dyr, ly), hy), dL = fminf(fmaxf(-dyr, ly), hy);
    float wR = fmaxf(taup - e * (dR * dR), 0.0f);
    float wL = fmaxf(taup - e * (dL * dL), 0.0f);
    float xr = mx + (sqrtf(wR / ca) - k * dR);
    float xl = mx - (sqrtf(wL / ca) + k * dL);
    float pr = 0x1p-6f + 0x1p-16f * (fabsf(mx) + fabsf(xr - mx));
    float pl = 0x1p-6f + 0x1p-16f * (fabsf(mx) + fabsf(xl - mx));
    /* NaN compares false in fmaxf/fminf: the rectangle's bound stays */
    float lo = fmaxf(ceilf((xl - pl) - 0.5f), (float)r[0]);
    float hi = fminf(floorf((xr + pr) - 0.5f), (float)r[1]);
    if (!(lo <= hi)) { *c0 = 1; *c1 = 0; return; }
    *c0 = (int)lo >> 4;
    *c1 = (int)hi >> 4;
}

/* Tiles per cell of a decision-mode pair: the row spans summed. */
static int64_t tiles32(const float *d, const int r[4]) {
    int64_t t = 0;
    for (int ty = r[2] >> 4; ty <= (r[3] >> 4); ty++) {
        int c0, c1;
        row_span32(d, r, ty, &c0, &c1);
        if (c0 <= c1) t += c1 - c0 + 1;
    }
    return t;
}

/* KD leaves whose box meets [lo, hi) per axis (half-open boxes). */
static void kd_collect(int nd, int depth, int L, const float *split, const float lo[3],
                       const float hi[3], uint64_t *mask) {
    int K = 1 << L;
    if (depth == L) { *mask |= 1ull << (nd - (K - 1)); return; }
    int a = depth % 3;
    if (lo[a] < split[nd]) kd_collect(2 * nd + 1, depth + 1, L, split, lo, hi, mask);
    if (hi[a] >= split[nd]) kd_collect(2 * nd + 2, depth + 1, L, split, lo, hi, mask);
}

/* Cell set of a Gaussian: the crossing point x(p) = o + z D(p) (Eq. 6's
 * x_i, read as the point of pixel p's ray on the plane through the centre
 * parallel to the image plane) is affine in the pixel coordinates, so over
 * the rectangle it stays inside the box spanned by the four corner
 * samples; that box, padded against fp32 rounding, is pushed down the
 * KD tree.  fp32 with a fixed operation order (mirror32).              */
static uint64_t cellset32(const P32 *p, const int rect[4], const Cam *c, int L, const float *split) {
    if (L == 0) return 1ull;
    float R[9];
    for (int k = 0; k < 9; k++) R[k] = (float)c->R[k];
    float fx = (float)c->fx, fy = (float)c->fy, cx = (float)c->cx, cy = (float)c->cy;
    float u0 = (float)rect[0] + 0.5f, u1 = (float)rect[1] + 0.5f;
    float v0 = (float)rect[2] + 0.5f, v1 = (float)rect[3] + 0.5f;
    float dx[2] = {(u0 - cx) / fx, (u1 - cx) / fx};
    float dy[2] = {(v0 - cy) / fy, (v1 - cy) / fy};
    float lo[3], hi[3];
    for (int a = 0; a < 3; a++) {
        float oa = (float)c->o[a];
        float mn = INFINITY, mxv = -INFINITY;
        for (int jy = 0; jy < 2; jy++) for (int jx = 0; jx < 2; jx++) {
            float Da = (R[a] * dx[jx] + R[3 + a] * dy[jy]) + R[6 + a];
            float xa = fmaf(p->z, Da, oa);
            mn = fminf(mn, xa); mxv = fmaxf(mxv, xa);
        }
        float mdx = fmaxf(fabsf(dx[0]), fabsf(dx[1])), mdy = fmaxf(fabsf(dy[0]), fabsf(dy[1]));
        float pad = 0x1p-16f * (fabsf(oa) + p->z * ((fabsf(R[a]) * mdx + fabsf(R[3 + a]) * mdy) + fabsf(R[6 + a])));
        lo[a] = mn - pad; hi[a] = mxv + pad;
    }
    uint64_t mask = 0;
    kd_collect(0, 0, L, split, lo, hi, &mask);
    return mask;
}
static uint64_t cellset64(const P64 *p, const int rect[4], const Cam *c, int L, const float *split) {
    if (L == 0) return 1ull;
    double dx[2] = {(rect[0] + 0.5 - c->cx) / c->fx, (rect[1] + 0.5 - c->cx) / c->fx};
    double dy[2] = {(rect[2] + 0.5 - c->cy) / c->fy, (rect[3] + 0.5 - c->cy) / c->fy};
    float lo[3], hi[3];
    for (int a = 0; a < 3; a++) {
        double mn = INFINITY, mxv = -INFINITY;
        for (int jy = 0; jy < 2; jy++) for (int jx = 0; jx < 2; jx++) {
            double Da = c->R[a] * dx[jx] + c->R[3 + a] * dy[jy] + c->R[6 + a];
            double xa = c->o[a] + p->z * Da;
            mn = fmin(mn, xa); mxv = fmax(mxv, xa);
        }
        double pad = 1e-9 * (fabs(c->o[a]) + p->z * (fabs(c->R[a]) + fabs(c->R[3 + a]) + fabs(c->R[6 + a])));
        lo[a] = (float)(mn - pad); hi[a] = (float)(mxv + pad);
        /* rounding to float: widen by one ulp each way */
        lo[a] = nextafterf(lo[a], -INFINITY); hi[a] = nextafterf(hi[a], INFINITY);
    }
    uint64_t mask = 0;
    kd_collect(0, 0, L, split, lo, hi, &mask);
    return mask;
}

static int popcount64(uint64_t x) { int c = 0; while (x) { x &= x - 1; c++; } return c; }

/* Which Gaussians a cell renders (cells):
 *   0  every Gaussian whose footprint can put its crossing point in the
 *      cell (the exact method: merged = plain);
 *   1  the paper's subsets N_k only (Sec. 3.3, the margin D_i): the set
 *      above restricted to the cells whose N_k holds the Gaussian (own_mask
 *      rows of ceil(K/32) words); contributions outside N_k are lost;
 *   2  exclusive subsets as in cell-based methods (Sec. 2): each Gaussian
 *      belongs to the cell of its centre only and renders its whole
 *      footprint there, without the indicator of Eq. 6 (center_cell).     */
static uint64_t own64(const uint32_t *own_mask, int K, int64_t i) {
    int W = (K + 31) / 32;
    uint64_t m = own_mask[i * W];
    if (W > 1) m |= (uint64_t)own_mask[i * W + 1] << 32;
    return m;
}

int orc_project(int64_t n, int D, const double *means, const double *log_scales, const double *quats,
                const double *opac, const double *sh, const double *cam, int L, const float *split,
                int mode, int cells, const int32_t *center_cell, const uint32_t *own_mask,
                float *dec32, double *val, int32_t *rect, uint8_t *vis, uint64_t *cellmask,
                uint32_t *count) {
    if (D < 0 || D > 3 || L < 0 || L > 6 || cells < 0 || cells > 2) return -1;
    if ((cells == 1 && !own_mask) || (cells == 2 && !center_cell)) return -1;
    Cam c; cam_unpack(cam, &c);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        P32 p32; P64 p64; int r[4] = {0, -1, 0, -1};
        proj32(n, means, log_scales, quats, opac, &c, i, &p32);
        proj64(n, D, means, log_scales, quats, opac, sh, &c, i, &p64);
        float *d = dec32 + 10 * i;
        d[0] = p32.mx; d[1] = p32.my; d[2] = p32.ca; d[3] = p32.cb; d[4] = p32.cc;
        d[5] = p32.tau; d[6] = p32.z; d[7] = p32.alpha; d[8] = p32.k; d[9] = p32.e;
        double *v = val + 12 * i;
        v[0] = p64.mx; v[1] = p64.my; v[2] = p64.ca; v[3] = p64.cb; v[4] = p64.cc;
        v[5] = p64.alpha; v[6] = p64.z; v[7] = p64.rgb[0]; v[8] = p64.rgb[1]; v[9] = p64.rgb[2];
        v[10] = p64.tau; v[11] = p64.det;
        int ok; uint64_t mask = 0;
        if (mode == 0) {
            ok = p32.vis && rect32(&p32, &c, r);
            /* the value path must exist wherever the decision path keeps a Gaussian */
            if (ok && !p64.vis) ok = 0;
            if (ok) mask = cellset32(&p32, r, &c, L, split);
        } else {
            ok = p64.vis && rect64(&p64, &c, r);
            if (ok) mask = cellset64(&p64, r, &c, L, split);
        }
        if (ok && cells == 1) mask &= own64(own_mask, 1 << L, i);
        if (ok && cells == 2) mask = 1ull << center_cell[i];
        vis[i] = (uint8_t)ok;
        for (int k = 0; k < 4; k++) rect[4 * i + k] = ok ? r[k] : 0;
        cellmask[i] = ok ? mask : 0;
        /* instances: cells x tiles; in decision mode the tiles are the row
         * spans of row_span32, in exact64 mode the whole rectangle */
        int64_t nt = mode == 0 ? tiles32(d, r) : (int64_t)((r[1] >> 4) - (r[0] >> 4) + 1) * ((r[3] >> 4) - (r[2] >> 4) + 1);
        count[i] = ok ? (uint32_t)(popcount64(mask) * nt) : 0;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* tile instance lists (for bit-exact checks of binning and sorting)   */
/* ------------------------------------------------------------------ */
typedef struct { uint32_t key; uint32_t zkey; uint32_t gid; } Inst;
static int cmp_inst(const void *a, const void *b) {
    const Inst *x = (const Inst *)a, *y = (const Inst *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->zkey != y->zkey) return x->zkey < y->zkey ? -1 : 1;
    return (x->gid > y->gid) - (x->gid < y->gid);
}

/* One instance per (Gaussian, cell in its cell set, 16x16 tile of its
 * rectangle inside the row spans of row_span32), keyed (tile << rank_bits
 * | rank of the cell in the view's order) and sorted by (key, depth, gid).
 * Depth is the fp32 camera z of the decision path; ties go to the smaller
 * gid.  Returns the count, or the negated required capacity if cap is too
 * small.                                                                */
int64_t orc_bins(int64_t n, const float *dec32, const int32_t *rect, const uint8_t *vis,
                 const uint64_t *cellmask, const int32_t *rank_of, int L, int tiles_x,
                 int64_t cap, uint32_t *keys, uint32_t *gids) {
    int K = 1 << L;
    int rb = L;
    int64_t tot = 0;
    for (int64_t i = 0; i < n; i++) {
        if (!vis[i]) continue;
        tot += (int64_t)popcount64(cellmask[i]) * tiles32(dec32 + 10 * i, rect + 4 * i);
    }
    if (tot > cap) return -tot;
    Inst *v = (Inst *)malloc(sizeof(Inst) * (tot > 0 ? tot : 1));
    int64_t m = 0;
    for (int64_t i = 0; i < n; i++) {
        if (!vis[i]) continue;
        float z = dec32[10 * i + 6];
        uint32_t zk; memcpy(&zk, &z, 4);
        for (int k = 0; k < K; k++) {
            if (!((cellmask[i] >> k) & 1)) continue;
            for (int ty = rect[4 * i + 2] >> 4; ty <= (rect[4 * i + 3] >> 4); ty++) {
                int c0, c1;
                row_span32(dec32 + 10 * i, rect + 4 * i, ty, &c0, &c1);
                for (int tx = c0; tx <= c1; tx++) {
                    uint32_t tile = (uint32_t)(ty * tiles_x + tx);
                    v[m].key = (tile << rb) | (uint32_t)rank_of[k];
                    v[m].zkey = zk; v[m].gid = (uint32_t)i; m++;
                }
            }
        }
    }
    qsort(v, (size_t)m, sizeof(Inst), cmp_inst);
    for (int64_t j = 0; j < m; j++) { keys[j] = v[j].key; gids[j] = v[j].gid; }
    free(v);
    return m;
}

/* ------------------------------------------------------------------ */
/* per-pixel rendering: Eq. 2 (plain), Eq. 3/4 (partials), Eq. 5 (merge) */
/* ------------------------------------------------------------------ */
typedef struct { double z; int64_t gid; int cell; double sigma, G; int clamped; double dx, dy; } Contrib;
static int cmp_contrib(const void *a, const void *b) {
    const Contrib *x = (const Contrib *)a, *y = (const Contrib *)b;
    if (x->z != y->z) return x->z < y->z ? -1 : 1;
    return (x->gid > y->gid) - (x->gid < y->gid);
}

typedef struct {
    int64_t n; const float *dec32; const double *val; const int32_t *rect; const uint8_t *vis;
    Cam c; int L; const float *split; int mode; const uint64_t *restrict_mask;
    int cells; const int32_t *center_cell; const uint32_t *own_mask;
} Scene;

/* The leaf containing point x (half-open boxes: coordinate >= split goes
 * right).  fp32 comparisons, as the splits are fp32.                   */
static int leaf_of32(const float x[3], int L, const float *split) {
    int nd = 0;
    for (int d = 0; d < L; d++) nd = (x[d % 3] >= split[nd]) ? 2 * nd + 2 : 2 * nd + 1;
    return nd - ((1 << L) - 1);
}
static int leaf_of64(const double x[3], int L, const float *split) {
    int nd = 0;
    for (int d = 0; d < L; d++) nd = (x[d % 3] >= (double)split[nd]) ? 2 * nd + 2 : 2 * nd + 1;
    return nd - ((1 << L) - 1);
}

/* Collect N_l for pixel (px, py): every visible Gaussian whose truncated
 * footprint contains the sample, with its cell k(i, p) and sigma, sorted
 * by depth (ties by gid).  Returns the count; *out is malloc'd.         */
static int64_t collect(const Scene *s, int px, int py, Contrib **out) {
    const Cam *c = &s->c;
    int64_t cap = 64, m = 0;
    Contrib *v = (Contrib *)malloc(sizeof(Contrib) * cap);
    float u32 = (float)px + 0.5f, v32 = (float)py + 0.5f;
    double u64 = px + 0.5, v64 = py + 0.5;
    /* ray direction D(p) in world coordinates */
    float R[9];
    for (int k = 0; k < 9; k++) R[k] = (float)c->R[k];
    float dxp = (u32 - (float)c->cx) / (float)c->fx, dyp = (v32 - (float)c->cy) / (float)c->fy;
    float D32[3];
    for (int a = 0; a < 3; a++) D32[a] = (R[a] * dxp + R[3 + a] * dyp) + R[6 + a];
    double dx64 = (u64 - c->cx) / c->fx, dy64 = (v64 - c->cy) / c->fy, D64[3];
    for (int a = 0; a < 3; a++) D64[a] = c->R[a] * dx64 + c->R[3 + a] * dy64 + c->R[6 + a];
    for (int64_t i = 0; i < s->n; i++) {
        if (!s->vis[i]) continue;
        const int32_t *r = s->rect + 4 * i;
        if (px < r[0] || px > r[1] || py < r[2] || py > r[3]) continue;
        const float *d = s->dec32 + 10 * i;
        const double *vv = s->val + 12 * i;
        int hit; double z; int cell;
        if (s->mode == 0) {
            float dx = u32 - d[0], dy = v32 - d[1];
            float u = fmaf(d[8], dy, dx);
            float d2 = fmaf(d[9] * dy, dy, (d[2] * u) * u);
            hit = (d2 <= d[5]);
            z = d[6];
            if (hit) {
                float x[3];
                for (int a = 0; a < 3; a++) x[a] = fmaf(d[6], D32[a], (float)c->o[a]);
                cell = leaf_of32(x, s->L, s->split);
            }
        } else {
            double dx = u64 - vv[0], dy = v64 - vv[1];
            double d2 = dx * (vv[2] * dx + 2 * vv[3] * dy) + vv[4] * dy * dy;
            hit = (d2 <= vv[10]);
            z = vv[6];
            if (hit) {
                double x[3];
                for (int a = 0; a < 3; a++) x[a] = c->o[a] + vv[6] * D64[a];
                cell = leaf_of64(x, s->L, s->split);
            }
        }
        if (!hit) continue;
        /* cell-based contrast mode: the centre's cell, no indicator */
        if (s->cells == 2) cell = s->center_cell[i];
        /* the paper's subsets: a contribution counts only if i is in N_k */
        if (s->cells == 1 && !((own64(s->own_mask, 1 << s->L, i) >> cell) & 1)) continue;
        /* diagnostic: keep only cells the Gaussian's emitted cell set names */
        if (s->restrict_mask && !((s->restrict_mask[i] >> cell) & 1)) continue;
        if (m == cap) { cap *= 2; v = (Contrib *)realloc(v, sizeof(Contrib) * cap); }
        /* value path in fp64 */
        double dx = u64 - vv[0], dy = v64 - vv[1];
        double d2 = vv[2] * dx * dx + 2 * vv[3] * dx * dy + vv[4] * dy * dy;
        double G = exp(-0.5 * d2);
        double sg = vv[5] * G;
        v[m].clamped = !(sg < 0.99);
        v[m].sigma = v[m].clamped ? 0.99 : sg;
        v[m].G = G; v[m].z = z; v[m].gid = i; v[m].cell = cell; v[m].dx = dx; v[m].dy = dy;
        m++;
    }
    qsort(v, (size_t)m, sizeof(Contrib), cmp_contrib);
    *out = v;
    return m;
}

/* Early termination floor: whatever the requested eps_T, a pixel stops in a
 * cell once its transmittance falls below 2^-100 (the contributions behind
 * it weigh less than that; the fp32 kernels keep T a normal number so that
 * their backward can recover the transmittance before each contribution). */
#define ORC_T_FLOOR 0x1p-100

/* Forward of one pixel.  Partial (C_k, T_k) of Eq. 3/4 over the
 * contributors whose crossing point lies in cell k, in depth order; the
 * cells are walked in the view's merge order (Eq. 5), so the product of
 * the finished cells' T_m times the current T_k is the transmittance of the
 * merged render.  Early termination is include-then-stop on that merged
 * transmittance at max(eps_T, ORC_T_FLOOR): the contributor that takes it
 * below the threshold is included, every later contributor of the pixel (in
 * this cell and in every cell after it) is not, and a cell reached after the
 * stop keeps C_k = 0, T_k = 1.  With the exact cell sets a ray meets the
 * cells in merge order, so this is the plain render's stop rule and merged =
 * plain holds with early termination too.  Merged colour by Eq. 5 plus
 * background; plain colour by Eq. 2 over all contributors (same stop rule on
 * its own transmittance).  `used` marks the contributors that were blended. */
static void pixel_forward(const Scene *s, const Contrib *v, int64_t m, const int32_t *order,
                          double eps_T, double *Ck, double *Tk, char *used, double out[3],
                          double *Tout, double plain[3], double *Tplain) {
    int K = 1 << s->L;
    if (eps_T < ORC_T_FLOOR) eps_T = ORC_T_FLOOR;
    for (int k = 0; k < K; k++) { Ck[3 * k] = Ck[3 * k + 1] = Ck[3 * k + 2] = 0; Tk[k] = 1; }
    for (int64_t j = 0; j < m; j++) used[j] = 0;
    double Tm = 1;   /* merged transmittance so far */
    int stopped = 0;
    for (int r = 0; r < K && !stopped; r++) {
        int k = order[r];
        for (int64_t j = 0; j < m; j++) {
            if (v[j].cell != k) continue;
            used[j] = 1;
            const double *rgb = s->val + 12 * v[j].gid + 7;
            for (int ch = 0; ch < 3; ch++) Ck[3 * k + ch] += rgb[ch] * v[j].sigma * Tk[k];
            Tk[k] *= (1 - v[j].sigma);
            Tm *= (1 - v[j].sigma);
            if (Tm < eps_T) { stopped = 1; break; }
        }
    }
    double C[3] = {0, 0, 0}, T = 1;
    for (int r = 0; r < K; r++) {
        int k = order[r];
        for (int ch = 0; ch < 3; ch++) C[ch] += T * Ck[3 * k + ch];
        T *= Tk[k];
    }
    for (int ch = 0; ch < 3; ch++) out[ch] = C[ch] + T * s->c.bg[ch];
    *Tout = T;
    double P[3] = {0, 0, 0}, TP = 1;
    for (int64_t j = 0; j < m; j++) {
        const double *rgb = s->val + 12 * v[j].gid + 7;
        for (int ch = 0; ch < 3; ch++) P[ch] += rgb[ch] * v[j].sigma * TP;
        TP *= (1 - v[j].sigma);
        if (TP < eps_T) break;
    }
    for (int ch = 0; ch < 3; ch++) plain[ch] = P[ch] + TP * s->c.bg[ch];
    *Tplain = TP;
}

/* mode: 0 mirror32 / 1 exact64 decisions; bit 1 (value 2) restricts each
 * Gaussian to the cells of its emitted cell set (restrict_mask).        */
/* cells: 0 / 1 / 2 as for orc_project (which Gaussians a cell renders). */
static int scene_init(Scene *s, int64_t n, const float *dec32, const double *val,
                      const int32_t *rect, const uint8_t *vis, const double *cam, int L,
                      const float *split, int mode, const uint64_t *restrict_mask, int cells,
                      const int32_t *center_cell, const uint32_t *own_mask) {
    s->n = n; s->dec32 = dec32; s->val = val; s->rect = rect; s->vis = vis;
    cam_unpack(cam, &s->c); s->L = L; s->split = split; s->mode = mode & 1;
    s->restrict_mask = (mode & 2) ? restrict_mask : NULL;
    s->cells = cells; s->center_cell = center_cell; s->own_mask = own_mask;
    if (cells < 0 || cells > 2 || (cells == 1 && !own_mask) || (cells == 2 && !center_cell)) return -1;
    return 0;
}

/* Render a list of pixels (pix = x0, y0, x1, y1, ...).
 * img[3]/Tf: merged (Eq. 5) + background; plain[3]/Tp: Eq. 2 + background;
 * partC[K][3]/partT[K]: per-cell partials indexed by cell id;
 * ncon: |N_l|.  Any output pointer may be NULL.                          */
int orc_render(int64_t n, const float *dec32, const double *val, const int32_t *rect,
               const uint8_t *vis, const double *cam, int L, const float *split,
               const int32_t *order, int mode, double eps_T, int64_t npix, const int32_t *pix,
               double *img, double *Tf, double *plain, double *Tp, double *partC,
               double *partT, int32_t *ncon, const uint64_t *cellmask, int cells,
               const int32_t *center_cell, const uint32_t *own_mask) {
    Scene s;
    if (scene_init(&s, n, dec32, val, rect, vis, cam, L, split, mode, cellmask, cells, center_cell, own_mask))
        return -1;
    int K = 1 << L;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < npix; q++) {
        Contrib *v; int64_t m = collect(&s, pix[2 * q], pix[2 * q + 1], &v);
        double Ck[3 * ORC_MAXK], Tk[ORC_MAXK], o3[3], To, p3[3], Tpl;
        char *used = (char *)malloc(m > 0 ? m : 1);
        pixel_forward(&s, v, m, order, eps_T, Ck, Tk, used, o3, &To, p3, &Tpl);
        if (img) for (int ch = 0; ch < 3; ch++) img[3 * q + ch] = o3[ch];
        if (Tf) Tf[q] = To;
        if (plain) for (int ch = 0; ch < 3; ch++) plain[3 * q + ch] = p3[ch];
        if (Tp) Tp[q] = Tpl;
        if (partC) for (int k = 0; k < 3 * K; k++) partC[3 * K * q + k] = Ck[k];
        if (partT) for (int k = 0; k < K; k++) partT[K * q + k] = Tk[k];
        if (ncon) ncon[q] = (int32_t)m;
        free(used); free(v);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* backward of the merged render (per pixel), to the 2D quantities      */
/* ------------------------------------------------------------------ */
/* For each pixel: the gradient of the merged image (dimg[3]) and of the
 * final transmittance (dTf) is sent through Eq. 5 to every cell's
 * (C_k, T_k), then through each cell's blend (Eq. 3/4) to sigma and the
 * colour of each processed contributor, then through
 * sigma = min(0.99, alpha exp(-d^2/2)) to alpha, the screen mean and the
 * conic.  g2d rows (per Gaussian, accumulated; caller zeroes):
 *   d mx, d my, d ca, d cb, d cc, d alpha, d r, d g, d b
 * (cb is the off-diagonal conic entry, which enters d^2 twice).          */
typedef struct { int64_t gid; double g[9]; } GRec;

int orc_render_bwd(int64_t n, const float *dec32, const double *val, const int32_t *rect,
                   const uint8_t *vis, const double *cam, int L, const float *split,
                   const int32_t *order, int mode, double eps_T, int64_t npix,
                   const int32_t *pix, const double *dimg, const double *dTf, double *g2d, int cells,
                   const int32_t *center_cell, const uint32_t *own_mask) {
    Scene s;
    if (scene_init(&s, n, dec32, val, rect, vis, cam, L, split, mode, NULL, cells, center_cell, own_mask))
        return -1;
    int K = 1 << L;
    GRec **recs = (GRec **)calloc(npix > 0 ? npix : 1, sizeof(GRec *));
    int64_t *nrec = (int64_t *)calloc(npix > 0 ? npix : 1, sizeof(int64_t));
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < npix; q++) {
        Contrib *v; int64_t m = collect(&s, pix[2 * q], pix[2 * q + 1], &v);
        double Ck[3 * ORC_MAXK], Tk[ORC_MAXK], o3[3], To, p3[3], Tpl;
        char *used = (char *)malloc(m > 0 ? m : 1);
        pixel_forward(&s, v, m, order, eps_T, Ck, Tk, used, o3, &To, p3, &Tpl);
        const double *g = dimg + 3 * q;
        double gT = dTf ? dTf[q] : 0.0;
        /* Eq. 5 backward: prefix P before each rank, suffix colour R and
         * transmittance Q after it.                                      */
        double dC[ORC_MAXK][3], dT[ORC_MAXK];
        double P[ORC_MAXK + 1];
        P[0] = 1;
        for (int r = 0; r < K; r++) P[r + 1] = P[r] * Tk[order[r]];
        double Rc[3] = {s.c.bg[0], s.c.bg[1], s.c.bg[2]}, Q = 1;
        for (int r = K - 1; r >= 0; r--) {
            int k = order[r];
            for (int ch = 0; ch < 3; ch++) dC[k][ch] = P[r] * g[ch];
            dT[k] = P[r] * (g[0] * Rc[0] + g[1] * Rc[1] + g[2] * Rc[2] + gT * Q);
            for (int ch = 0; ch < 3; ch++) Rc[ch] = Ck[3 * k + ch] + Tk[k] * Rc[ch];
            Q *= Tk[k];
        }
        /* Eq. 3/4 backward per cell: transmittance before each processed
         * contributor and the colour sum S of those behind it.           */
        GRec *out = (GRec *)malloc(sizeof(GRec) * (m > 0 ? m : 1));
        int64_t no = 0;
        double *Tbef = (double *)malloc(sizeof(double) * (m > 0 ? m : 1));
        double Tc[ORC_MAXK];
        for (int k = 0; k < K; k++) Tc[k] = 1;
        for (int64_t j = 0; j < m; j++) if (used[j]) { Tbef[j] = Tc[v[j].cell]; Tc[v[j].cell] *= 1 - v[j].sigma; }
        double S[ORC_MAXK][3];
        memset(S, 0, sizeof(S));
        for (int64_t j = m - 1; j >= 0; j--) {
            if (!used[j]) continue;
            int k = v[j].cell;
            const double *rgb = s.val + 12 * v[j].gid + 7;
            double sg = v[j].sigma, T = Tbef[j];
            double dsg = 0;
            for (int ch = 0; ch < 3; ch++) dsg += dC[k][ch] * (rgb[ch] * T - S[k][ch] / (1 - sg));
            dsg += dT[k] * (-Tk[k] / (1 - sg));
            GRec *o = &out[no++];
            memset(o, 0, sizeof(*o));
            o->gid = v[j].gid;
            for (int ch = 0; ch < 3; ch++) o->g[6 + ch] = sg * T * dC[k][ch];
            if (!v[j].clamped) {
                const double *vv = s.val + 12 * v[j].gid;
                double G = v[j].G, al = vv[5];
                double dd2 = dsg * al * G * (-0.5);
                double dx = v[j].dx, dy = v[j].dy;
                o->g[5] = dsg * G;
                o->g[0] = dd2 * (-2.0) * (vv[2] * dx + vv[3] * dy);
                o->g[1] = dd2 * (-2.0) * (vv[3] * dx + vv[4] * dy);
                o->g[2] = dd2 * dx * dx;
                o->g[3] = dd2 * 2.0 * dx * dy;
                o->g[4] = dd2 * dy * dy;
            }
            for (int ch = 0; ch < 3; ch++) S[k][ch] += rgb[ch] * sg * T;
        }
        recs[q] = out; nrec[q] = no;
        free(Tbef); free(used); free(v);
    }
    /* fixed-order accumulation: pixels in list order */
    for (int64_t q = 0; q < npix; q++) {
        for (int64_t j = 0; j < nrec[q]; j++)
            for (int c = 0; c < 9; c++) g2d[9 * recs[q][j].gid + c] += recs[q][j].g[c];
        free(recs[q]);
    }
    free(recs); free(nrec);
    return 0;
}

/* ------------------------------------------------------------------ */
/* projection backward (fp64)                                           */
/* ------------------------------------------------------------------ */
/* Chain rule from the 2D quantities (screen mean, conic, alpha, colour)
 * back to the parameters.  Derivatives are exact: zero through the colour
 * clamp, through the clamp of the EWA Jacobian's x/z, y/z (where the
 * clamped value is proportional to z), and for culled Gaussians.
 * Gradients are written (not accumulated) in the parameter layout.      */
int orc_project_bwd(int64_t n, int D, const double *means, const double *log_scales,
                    const double *quats, const double *opac, const double *sh, const double *cam,
                    const uint8_t *vis, const double *g2d, double *g_means, double *g_ls,
                    double *g_q, double *g_op, double *g_sh) {
    Cam c; cam_unpack(cam, &c);
    int nc = (D + 1) * (D + 1);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        for (int a = 0; a < 3; a++) { g_means[a * n + i] = 0; g_ls[a * n + i] = 0; }
        for (int a = 0; a < 4; a++) g_q[a * n + i] = 0;
        g_op[i] = 0;
        for (int j = 0; j < 3 * nc; j++) g_sh[j * n + i] = 0;
        if (!vis[i]) continue;
        const double *g = g2d + 9 * i;
        double mu[3] = {means[i], means[n + i], means[2 * n + i]};
        double s[3] = {exp(log_scales[i]), exp(log_scales[n + i]), exp(log_scales[2 * n + i])};
        double alpha = 1.0 / (1.0 + exp(-opac[i]));
        double q4[4] = {quats[i], quats[n + i], quats[2 * n + i], quats[3 * n + i]};
        double qn = sqrt(q4[0] * q4[0] + q4[1] * q4[1] + q4[2] * q4[2] + q4[3] * q4[3]);
        double w = q4[0] / qn, x = q4[1] / qn, y = q4[2] / qn, z = q4[3] / qn;
        double Rq[3][3] = {
            {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
            {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
            {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
        double M[3][3], S[3][3];
        for (int a = 0; a < 3; a++) for (int b = 0; b < 3; b++) M[a][b] = Rq[a][b] * s[b];
        for (int a = 0; a < 3; a++) for (int b = 0; b < 3; b++)
            S[a][b] = M[a][0] * M[b][0] + M[a][1] * M[b][1] + M[a][2] * M[b][2];
        double t[3];
        for (int a = 0; a < 3; a++)
            t[a] = c.R[3 * a] * mu[0] + c.R[3 * a + 1] * mu[1] + c.R[3 * a + 2] * mu[2] + c.t[a];
        double zc = t[2];
        double gx = 1.3 * (fmax(c.cx, c.W - c.cx) / c.fx);
        double gy = 1.3 * (fmax(c.cy, c.H - c.cy) / c.fy);
        double xz = t[0] / zc, yz = t[1] / zc;
        int clx = (xz < -gx) ? -1 : (xz > gx ? 1 : 0);
        int cly = (yz < -gy) ? -1 : (yz > gy ? 1 : 0);
        double xg = clx ? clx * gx * zc : t[0];
        double yg = cly ? cly * gy * zc : t[1];
        double J[2][3] = {{c.fx / zc, 0, -c.fx * xg / (zc * zc)}, {0, c.fy / zc, -c.fy * yg / (zc * zc)}};
        double T[2][3];
        for (int a = 0; a < 2; a++) for (int b = 0; b < 3; b++)
            T[a][b] = J[a][0] * c.R[b] + J[a][1] * c.R[3 + b] + J[a][2] * c.R[6 + b];
        double S2[2][2];
        for (int a = 0; a < 2; a++) for (int b = 0; b < 2; b++) {
            double v = 0;
            for (int k = 0; k < 3; k++) for (int l = 0; l < 3; l++) v += T[a][k] * S[k][l] * T[b][l];
            S2[a][b] = v;
        }
        S2[0][0] += 0.3; S2[1][1] += 0.3;
        double det = S2[0][0] * S2[1][1] - S2[0][1] * S2[1][0];
        double Cn[2][2] = {{S2[1][1] / det, -S2[0][1] / det}, {-S2[1][0] / det, S2[0][0] / det}};
        /* conic -> screen covariance: G_S2 = -Cn G_C Cn */
        double GC[2][2] = {{g[2], 0.5 * g[3]}, {0.5 * g[3], g[4]}};
        double GS2[2][2];
        for (int a = 0; a < 2; a++) for (int b = 0; b < 2; b++) {
            double v = 0;
            for (int k = 0; k < 2; k++) for (int l = 0; l < 2; l++) v += Cn[a][k] * GC[k][l] * Cn[l][b];
            GS2[a][b] = -v;
        }
        /* S2 = T S T^T: G_T = 2 G_S2 T S, G_S = T^T G_S2 T */
        double GT[2][3], GS[3][3];
        for (int a = 0; a < 2; a++) for (int b = 0; b < 3; b++) {
            double v = 0;
            for (int k = 0; k < 2; k++) for (int l = 0; l < 3; l++) v += GS2[a][k] * T[k][l] * S[l][b];
            GT[a][b] = 2 * v;
        }
        for (int a = 0; a < 3; a++) for (int b = 0; b < 3; b++) {
            double v = 0;
            for (int k = 0; k < 2; k++) for (int l = 0; l < 2; l++) v += T[k][a] * GS2[k][l] * T[l][b];
            GS[a][b] = v;
        }
        /* T = J R: G_J = G_T R^T */
        double GJ[2][3];
        for (int a = 0; a < 2; a++) for (int b = 0; b < 3; b++)
            GJ[a][b] = GT[a][0] * c.R[3 * b] + GT[a][1] * c.R[3 * b + 1] + GT[a][2] * c.R[3 * b + 2];
        double gt[3] = {0, 0, 0};
        double z2 = zc * zc, z3 = z2 * zc;
        gt[2] += GJ[0][0] * (-c.fx / z2) + GJ[1][1] * (-c.fy / z2);
        gt[2] += GJ[0][2] * (2 * c.fx * xg / z3) + GJ[1][2] * (2 * c.fy * yg / z3);
        double gxg = GJ[0][2] * (-c.fx / z2), gyg = GJ[1][2] * (-c.fy / z2);
        if (clx) gt[2] += gxg * clx * gx; else gt[0] += gxg;
        if (cly) gt[2] += gyg * cly * gy; else gt[1] += gyg;
        /* screen mean */
        gt[0] += g[0] * c.fx / zc; gt[2] += -g[0] * c.fx * t[0] / z2;
        gt[1] += g[1] * c.fy / zc; gt[2] += -g[1] * c.fy * t[1] / z2;
        double gmu[3];
        for (int a = 0; a < 3; a++) gmu[a] = c.R[a] * gt[0] + c.R[3 + a] * gt[1] + c.R[6 + a] * gt[2];
        /* colour */
        double d[3] = {mu[0] - c.o[0], mu[1] - c.o[1], mu[2] - c.o[2]};
        double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double dir[3] = {d[0] / dn, d[1] / dn, d[2] / dn};
        double Y[16], dY[48];
        orc_sh_basis(D, dir, Y, dY);
        double gdir[3] = {0, 0, 0};
        for (int ch = 0; ch < 3; ch++) {
            double v = 0.5;
            for (int j = 0; j < nc; j++) v += sh[(3 * j + ch) * n + i] * Y[j];
            if (!(v > 0)) continue;
            double gc = g[6 + ch];
            for (int j = 0; j < nc; j++) {
                g_sh[(3 * j + ch) * n + i] = Y[j] * gc;
                double f = sh[(3 * j + ch) * n + i];
                for (int a = 0; a < 3; a++) gdir[a] += f * dY[3 * j + a] * gc;
            }
        }
        double dg = dir[0] * gdir[0] + dir[1] * gdir[1] + dir[2] * gdir[2];
        for (int a = 0; a < 3; a++) gmu[a] += (gdir[a] - dir[a] * dg) / dn;
        for (int a = 0; a < 3; a++) g_means[a * n + i] = gmu[a];
        /* opacity */
        g_op[i] = g[5] * alpha * (1 - alpha);
        /* S = M M^T: G_M = 2 G_S M;  M = Rq diag(s) */
        double GM[3][3];
        for (int a = 0; a < 3; a++) for (int b = 0; b < 3; b++)
            GM[a][b] = 2 * (GS[a][0] * M[0][b] + GS[a][1] * M[1][b] + GS[a][2] * M[2][b]);
        double GR[3][3];
        for (int b = 0; b < 3; b++) {
            double gs = 0;
            for (int a = 0; a < 3; a++) { gs += GM[a][b] * Rq[a][b]; GR[a][b] = GM[a][b] * s[b]; }
            g_ls[b * n + i] = gs * s[b];
        }
        /* rotation entries -> unit quaternion (w, x, y, z) */
        double gw = 0, gx_ = 0, gy_ = 0, gz_ = 0;
        gy_ += GR[0][0] * (-4 * y); gz_ += GR[0][0] * (-4 * z);
        gw += GR[0][1] * (-2 * z); gx_ += GR[0][1] * (2 * y); gy_ += GR[0][1] * (2 * x); gz_ += GR[0][1] * (-2 * w);
        gw += GR[0][2] * (2 * y); gx_ += GR[0][2] * (2 * z); gy_ += GR[0][2] * (2 * w); gz_ += GR[0][2] * (2 * x);
        gw += GR[1][0] * (2 * z); gx_ += GR[1][0] * (2 * y); gy_ += GR[1][0] * (2 * x); gz_ += GR[1][0] * (2 * w);
        gx_ += GR[1][1] * (-4 * x); gz_ += GR[1][1] * (-4 * z);
        gw += GR[1][2] * (-2 * x); gx_ += GR[1][2] * (-2 * w); gy_ += GR[1][2] * (2 * z); gz_ += GR[1][2] * (2 * y);
        gw += GR[2][0] * (-2 * y); gx_ += GR[2][0] * (2 * z); gy_ += GR[2][0] * (-2 * w); gz_ += GR[2][0] * (2 * x);
        gw += GR[2][1] * (2 * x); gx_ += GR[2][1] * (2 * w); gy_ += GR[2][1] * (2 * z); gz_ += GR[2][1] * (2 * y);
        gx_ += GR[2][2] * (-4 * x); gy_ += GR[2][2] * (-4 * y);
        double qh[4] = {w, x, y, z}, gqh[4] = {gw, gx_, gy_, gz_};
        double dot = qh[0] * gqh[0] + qh[1] * gqh[1] + qh[2] * gqh[2] + qh[3] * gqh[3];
        for (int a = 0; a < 4; a++) g_q[a * n + i] = (gqh[a] - qh[a] * dot) / qn;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* loss: L1 + w (1 - SSIM), fp64                                        */
/* ------------------------------------------------------------------ */
/* L1 = mean |x - y| over C*H*W (sign(0) = 0).  SSIM per channel with an
 * 11x11 Gaussian window (std 1.5, normalised to sum 1), zero padding
 * ("same" size), C1 = 0.01^2, C2 = 0.03^2, averaged over C*H*W.
 * Direct 2D convolutions (no separable filtering).                       */
static void conv2d(int H, int W, const double *w11, const double *src, double *dst) {
    for (int y = 0; y < H; y++) for (int x = 0; x < W; x++) {
        double acc = 0;
        for (int dy = -5; dy <= 5; dy++) for (int dx = -5; dx <= 5; dx++) {
            int yy = y + dy, xx = x + dx;
            if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
            acc += w11[(dy + 5) * 11 + (dx + 5)] * src[yy * W + xx];
        }
        dst[y * W + x] = acc;
    }
}

int orc_loss(int C, int H, int W, const double *img, const double *tgt, double ssim_w,
             double *loss, double *dimg) {
    double g1[11], gs = 0, w11[121];
    for (int i = 0; i < 11; i++) { g1[i] = exp(-((i - 5) * (i - 5)) / (2 * 1.5 * 1.5)); gs += g1[i]; }
    for (int i = 0; i < 11; i++) for (int j = 0; j < 11; j++) w11[i * 11 + j] = g1[i] * g1[j] / (gs * gs);
    const double C1 = 0.01 * 0.01, C2 = 0.03 * 0.03;
    double N = (double)C * H * W, l1 = 0, ssim = 0;
    int64_t HW = (int64_t)H * W;
    for (int64_t k = 0; k < C * HW; k++) {
        double d = img[k] - tgt[k];
        l1 += fabs(d);
        dimg[k] = ((d > 0) - (d < 0)) / N;
    }
    if (ssim_w != 0) {
        double *buf = (double *)malloc(sizeof(double) * HW * 12);
        double *xx = buf, *yy = buf + HW, *xy = buf + 2 * HW, *mx = buf + 3 * HW, *my = buf + 4 * HW;
        double *exx = buf + 5 * HW, *eyy = buf + 6 * HW, *exy = buf + 7 * HW;
        double *gmx = buf + 8 * HW, *gxx = buf + 9 * HW, *gxy = buf + 10 * HW, *tmp = buf + 11 * HW;
        for (int ch = 0; ch < C; ch++) {
            const double *x = img + ch * HW, *y = tgt + ch * HW;
            for (int64_t k = 0; k < HW; k++) { xx[k] = x[k] * x[k]; yy[k] = y[k] * y[k]; xy[k] = x[k] * y[k]; }
            conv2d(H, W, w11, x, mx); conv2d(H, W, w11, y, my);
            conv2d(H, W, w11, xx, exx); conv2d(H, W, w11, yy, eyy); conv2d(H, W, w11, xy, exy);
            for (int64_t k = 0; k < HW; k++) {
                double A1 = 2 * mx[k] * my[k] + C1, A2 = 2 * (exy[k] - mx[k] * my[k]) + C2;
                double B1 = mx[k] * mx[k] + my[k] * my[k] + C1;
                double B2 = (exx[k] - mx[k] * mx[k]) + (eyy[k] - my[k] * my[k]) + C2;
                double Nn = A1 * A2, Dd = B1 * B2;
                ssim += Nn / Dd;
                /* partial derivatives of S = Nn/Dd w.r.t. mu_x, E[x^2], E[xy] */
                double dN_dmx = 2 * my[k] * A2 + A1 * (-2 * my[k]);
                double dD_dmx = 2 * mx[k] * B2 + B1 * (-2 * mx[k]);
                gmx[k] = (dN_dmx * Dd - Nn * dD_dmx) / (Dd * Dd);
                gxx[k] = -Nn * B1 / (Dd * Dd);
                gxy[k] = 2 * A1 / Dd;
            }
            /* adjoint of the symmetric zero-padded convolution is itself */
            double sc = -ssim_w / N;
            conv2d(H, W, w11, gmx, tmp);
            for (int64_t k = 0; k < HW; k++) dimg[ch * HW + k] += sc * tmp[k];
            conv2d(H, W, w11, gxx, tmp);
            for (int64_t k = 0; k < HW; k++) dimg[ch * HW + k] += sc * 2 * x[k] * tmp[k];
            conv2d(H, W, w11, gxy, tmp);
            for (int64_t k = 0; k < HW; k++) dimg[ch * HW + k] += sc * y[k] * tmp[k];
        }
        free(buf);
    }
    *loss = l1 / N + (ssim_w != 0 ? ssim_w * (1 - ssim / N) : 0);
    return 0;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the parallel loops from now on (results do not depend on it:
 * every reduction above runs in a fixed order). */
void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
