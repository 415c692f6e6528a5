/*
 * rn_oracle.c -- CPU FP64 reference for steady flow through a random network.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the parity oracle: only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark load it.
 * The solver library shares no code, header, table or helper with it.
 *
 * What it computes (Dashtian & Sahimi, Sec. II):
 *   - a square (2D) or simple-cubic (3D) lattice whose bonds carry
 *     conductances g_ij >= 0 (g = 0: removed bond, percolation dilution of
 *     Sec. V-VI);
 *   - mass balance sum_j g_ij (P_j - P_i) = 0 at every interior node (Eq. 3,
 *     G P = b), with the pressure fixed to 1 on the inlet face (first node
 *     plane along the flow axis) and 0 on the outlet face (last plane), and no
 *     flow through the side faces;
 *   - the total flux Q and Darcy's K = (Q / S) (mu L / dP) (Eq. 4) with
 *     mu = dP = 1, L = n_axis - 1 bond lengths and S = number of node lines
 *     crossing a section (product of the other extents).
 *
 * Interior nodes that are not connected, through occupied interior bonds, to
 * both faces carry no flow; they are excluded from the unknowns (the "live"
 * set). The solve is Jacobi-preconditioned conjugate gradients (Sec. II-IV;
 * the CG method of the paper's ref. [57], Barrett et al., Templates), run in
 * FP64 with pairwise-summed dot products.
 *
 * Lattice convention: node i = x + nx*(y + ny*z); g[k][i] is the bond from i
 * to i + e_k (k = 0,1,2 for x,y,z); entries whose neighbour is off the
 * lattice are ignored.
 *
 * Side boundaries: no flow by default. With `periodic` set, every direction
 * other than the flow axis wraps around (Sec. II imposes the pressure drop
 * along one direction and periodic conditions along the other): the entry
 * g[k][i] on the last plane along k is then the bond to the first plane. A
 * direction of extent 1 has no bonds along it either way.
 *
 * Parity status of each function: every function here is pinned by the CPU
 * tests (closed forms, dense direct solves, brute-force connectivity, planar
 * duality, conservation identities; for periodic sides also a hand-solved
 * path across the wrap and invariance under translation along a wrapped
 * direction); iteration counts are reported but parity-unpinned (the paper
 * prints none). The backbone (rno_backbone) is pinned by a hand-built
 * network, a brute-force vertex-cut check on tiny lattices and the physics of
 * a dense direct solve (no current off the backbone).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define RNO_OK 0
#define RNO_EINVAL (-1)
#define RNO_ENOMEM (-2)
#define RNO_ENOCONV (-3)
#define RNO_ENUMERIC (-4)

typedef struct {
    int32_t status, converged;
    double Q_in, Q_out, G, K, rel_resid;
    int64_t iters, n_live;
} rno_result;

typedef struct {
    int dim, axis;
    int wrap[3];       /* direction k wraps around (periodic sides, extent >= 2) */
    int64_t n[3];      /* nx, ny, nz */
    int64_t stride[3]; /* 1, nx, nx*ny */
    int64_t N;
    const double *g[3];
} lat_t;

/* ------------------------------------------------------------------ lattice */

static int64_t coord(const lat_t *L, int64_t i, int k) { return (i / L->stride[k]) % L->n[k]; }

/* Neighbour across direction k and sign s (+1/-1) of the node with index i
 * and coordinates c; returns -1 when there is none. *gij receives the bond
 * conductance (0 when there is no neighbour). Across a periodic direction the
 * last plane's +1 neighbour is the first plane, through the last plane's own
 * bond entry. */
static int64_t nbr_at(const lat_t *L, const int64_t c[3], int64_t i, int k, int s, double *gij)
{
    const int64_t n = L->n[k], st = L->stride[k];
    if (s > 0) {
        if (c[k] + 1 < n) { *gij = L->g[k][i]; return i + st; }
        if (L->wrap[k]) { *gij = L->g[k][i]; return i - (n - 1) * st; }
        *gij = 0.0;
        return -1;
    }
    if (c[k] > 0) { *gij = L->g[k][i - st]; return i - st; }
    if (L->wrap[k]) { *gij = L->g[k][i + (n - 1) * st]; return i + (n - 1) * st; }
    *gij = 0.0;
    return -1;
}

static int64_t nbr(const lat_t *L, int64_t i, int k, int s, double *gij)
{
    const int64_t c[3] = {coord(L, i, 0), coord(L, i, 1), coord(L, i, 2)};
    return nbr_at(L, c, i, k, s, gij);
}

/* Face classification along the flow axis: 0 interior, 1 inlet, 2 outlet. */
static int face_of(const lat_t *L, int64_t i)
{
    int64_t c = coord(L, i, L->axis);
    if (c == 0) return 1;
    if (c == L->n[L->axis] - 1) return 2;
    return 0;
}

static int setup(lat_t *L, int dim, int64_t nx, int64_t ny, int64_t nz, int axis, int periodic,
                 const double *g0, const double *g1, const double *g2)
{
    if (dim != 2 && dim != 3) return RNO_EINVAL;
    if (nx < 1 || ny < 1 || nz < 1) return RNO_EINVAL;
    if (dim == 2 && nz != 1) return RNO_EINVAL;
    if (axis < 0 || axis >= dim) return RNO_EINVAL;
    L->dim = dim;
    L->axis = axis;
    L->n[0] = nx; L->n[1] = ny; L->n[2] = nz;
    L->stride[0] = 1; L->stride[1] = nx; L->stride[2] = nx * ny;
    L->N = nx * ny * nz;
    if (L->n[axis] < 2) return RNO_EINVAL;
    L->g[0] = g0; L->g[1] = g1; L->g[2] = (dim == 3) ? g2 : NULL;
    if (periodic != 0 && periodic != 1) return RNO_EINVAL;
    for (int k = 0; k < 3; ++k) L->wrap[k] = periodic && k < dim && k != axis && L->n[k] >= 2;
    for (int k = 0; k < dim; ++k) {
        if (!L->g[k]) return RNO_EINVAL;
        for (int64_t i = 0; i < L->N; ++i) {
            if (coord(L, i, k) + 1 >= L->n[k] && !L->wrap[k]) continue; /* off-lattice entry: ignored */
            double v = L->g[k][i];
            if (!(v >= 0.0) || isinf(v)) return RNO_EINVAL;  /* negative, NaN or Inf */
        }
    }
    return RNO_OK;
}

/* ------------------------------------------------------- connectivity (BFS) */
/*
 * Mask byte per node: bit0 = the node's interior component has an occupied
 * bond to an inlet-face node, bit1 = same for the outlet face, bit2 = face
 * node. Inlet face = 5, outlet face = 6, live interior = 3. Paths run only
 * through occupied interior-interior bonds; face nodes are never traversed.
 */
static int64_t bfs_from_face(const lat_t *L, int which, uint8_t bit, uint8_t *mask, int64_t *queue)
{
    int64_t head = 0, tail = 0;
    for (int64_t i = 0; i < L->N; ++i) {
        if (face_of(L, i) != 0 || (mask[i] & bit)) continue;
        for (int k = 0; k < L->dim; ++k)
            for (int s = -1; s <= 1; s += 2) {
                double gij;
                int64_t j = nbr(L, i, k, s, &gij);
                if (j >= 0 && gij > 0.0 && face_of(L, j) == which && !(mask[i] & bit)) {
                    mask[i] |= bit;
                    queue[tail++] = i;
                }
            }
    }
    while (head < tail) {
        int64_t i = queue[head++];
        for (int k = 0; k < L->dim; ++k)
            for (int s = -1; s <= 1; s += 2) {
                double gij;
                int64_t j = nbr(L, i, k, s, &gij);
                if (j < 0 || !(gij > 0.0) || face_of(L, j) != 0 || (mask[j] & bit)) continue;
                mask[j] |= bit;
                queue[tail++] = j;
            }
    }
    return tail;
}

static int mask_bfs(const lat_t *L, uint8_t *mask, int64_t *n_live)
{
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(L->N > 0 ? L->N : 1));
    if (!queue) return RNO_ENOMEM;
    memset(mask, 0, (size_t)L->N);
    bfs_from_face(L, 1, 1u, mask, queue);
    bfs_from_face(L, 2, 2u, mask, queue);
    free(queue);
    int64_t live = 0;
    for (int64_t i = 0; i < L->N; ++i) {
        int f = face_of(L, i);
        if (f == 1) mask[i] = 5;
        else if (f == 2) mask[i] = 6;
        else if (mask[i] == 3) ++live;
    }
    if (n_live) *n_live = live;
    return RNO_OK;
}

int rno_mask_bfs(int dim, int64_t nx, int64_t ny, int64_t nz, int axis, int periodic,
                 const double *g0, const double *g1, const double *g2,
                 uint8_t *mask_out, int64_t *n_live_out)
{
    lat_t L;
    int st = setup(&L, dim, nx, ny, nz, axis, periodic, g0, g1, g2);
    if (st) return st;
    return mask_bfs(&L, mask_out, n_live_out);
}

/* ------------------------------------------- connectivity (union-find, second) */
/* An independent route to the same mask: sequential union by size with path
 * compression over occupied interior-interior bonds, then per-component face
 * flags. Used by the tests to cross-check the BFS. */
static int64_t uf_find(int64_t *par, int64_t a)
{
    int64_t r = a;
    while (par[r] != r) r = par[r];
    while (par[a] != r) { int64_t nx_ = par[a]; par[a] = r; a = nx_; }
    return r;
}

int rno_mask_uf(int dim, int64_t nx, int64_t ny, int64_t nz, int axis, int periodic,
                const double *g0, const double *g1, const double *g2,
                uint8_t *mask_out, int64_t *n_live_out)
{
    lat_t L;
    int st = setup(&L, dim, nx, ny, nz, axis, periodic, g0, g1, g2);
    if (st) return st;
    int64_t *par = (int64_t *)malloc(sizeof(int64_t) * (size_t)L.N);
    int64_t *sz = (int64_t *)malloc(sizeof(int64_t) * (size_t)L.N);
    uint8_t *flag = (uint8_t *)calloc((size_t)L.N, 1);
    if (!par || !sz || !flag) { free(par); free(sz); free(flag); return RNO_ENOMEM; }
    for (int64_t i = 0; i < L.N; ++i) { par[i] = i; sz[i] = 1; }
    for (int64_t i = 0; i < L.N; ++i) {
        if (face_of(&L, i) != 0) continue;
        for (int k = 0; k < L.dim; ++k) {
            double gij;
            int64_t j = nbr(&L, i, k, +1, &gij);
            if (j < 0 || !(gij > 0.0) || face_of(&L, j) != 0) continue;
            int64_t a = uf_find(par, i), b = uf_find(par, j);
            if (a == b) continue;
            if (sz[a] < sz[b]) { int64_t t = a; a = b; b = t; }
            par[b] = a;
            sz[a] += sz[b];
        }
    }
    for (int64_t i = 0; i < L.N; ++i) {
        if (face_of(&L, i) != 0) continue;
        for (int k = 0; k < L.dim; ++k)
            for (int s = -1; s <= 1; s += 2) {
                double gij;
                int64_t j = nbr(&L, i, k, s, &gij);
                if (j < 0 || !(gij > 0.0)) continue;
                int f = face_of(&L, j);
                if (f) flag[uf_find(par, i)] |= (uint8_t)f; /* inlet 1 -> bit0, outlet 2 -> bit1 */
            }
    }
    int64_t live = 0;
    for (int64_t i = 0; i < L.N; ++i) {
        int f = face_of(&L, i);
        if (f == 1) mask_out[i] = 5;
        else if (f == 2) mask_out[i] = 6;
        else {
            mask_out[i] = flag[uf_find(par, i)];
            if (mask_out[i] == 3) ++live;
        }
    }
    if (n_live_out) *n_live_out = live;
    free(par); free(sz); free(flag);
    return RNO_OK;
}

/* ---------------------------------------------------------------- FP64 linear algebra */

/* Pairwise (recursive halving) dot product: error grows like log n. */
static double pdot(const double *a, const double *b, int64_t n)
{
    if (n <= 64) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
        return s;
    }
    int64_t h = n / 2;
    return pdot(a, b, h) + pdot(a + h, b + h, n - h);
}

/* Operator of Eq. 3 restricted to the live set:
 *   (A v)_i = d_i v_i - sum_{j live neighbour} g_ij v_j   for live i, 0 otherwise,
 * with d_i the sum of the conductances of all occupied bonds at i. */
static void apply_A(const lat_t *L, const uint8_t *mask, const double *d, const double *v, double *out)
{
    int64_t c[3];
    for (c[2] = 0; c[2] < L->n[2]; ++c[2])
        for (c[1] = 0; c[1] < L->n[1]; ++c[1])
            for (c[0] = 0; c[0] < L->n[0]; ++c[0]) {
                const int64_t i = c[0] + L->stride[1] * c[1] + L->stride[2] * c[2];
                if (mask[i] != 3) { out[i] = 0.0; continue; }
                double s = d[i] * v[i];
                for (int k = 0; k < L->dim; ++k)
                    for (int sg = -1; sg <= 1; sg += 2) {
                        double gij;
                        const int64_t j = nbr_at(L, c, i, k, sg, &gij);
                        if (j >= 0 && mask[j] == 3) s -= gij * v[j];
                    }
                out[i] = s;
            }
}

/* Diagonal d_i and right-hand side b_i (inflow from inlet-face neighbours at
 * unit pressure) for live nodes; zero elsewhere. */
static void assemble(const lat_t *L, const uint8_t *mask, double *d, double *b)
{
    for (int64_t i = 0; i < L->N; ++i) {
        d[i] = 0.0;
        b[i] = 0.0;
        if (mask[i] != 3) continue;
        for (int k = 0; k < L->dim; ++k)
            for (int sg = -1; sg <= 1; sg += 2) {
                double gij;
                int64_t j = nbr(L, i, k, sg, &gij);
                if (j < 0 || !(gij > 0.0)) continue;
                d[i] += gij;
                if (face_of(L, j) == 1) b[i] += gij;
            }
    }
}

/* Full pressure field from the live solution x: faces at 1 / 0, live nodes x,
 * dead interior nodes 1 when connected to the inlet only, else 0. */
static void fill_pressure(const lat_t *L, const uint8_t *mask, const double *x, double *P)
{
    for (int64_t i = 0; i < L->N; ++i) {
        uint8_t m = mask[i];
        if (m == 5) P[i] = 1.0;
        else if (m == 6) P[i] = 0.0;
        else if (m == 3) P[i] = x[i];
        else if (m == 1) P[i] = 1.0;
        else P[i] = 0.0;
    }
}

/* Fluxes of a full pressure field P: Q_in = inflow through inlet-face bonds
 * into the interior plus direct inlet-outlet bonds; Q_out = outflow into the
 * outlet face plus the same direct bonds. */
static void face_fluxes(const lat_t *L, const double *P, double *Qin, double *Qout)
{
    double qi = 0.0, qo = 0.0;
    for (int64_t i = 0; i < L->N; ++i) {
        int fi = face_of(L, i);
        for (int k = 0; k < L->dim; ++k)
            for (int sg = -1; sg <= 1; sg += 2) {
                double gij;
                int64_t j = nbr(L, i, k, sg, &gij);
                if (j < 0 || !(gij > 0.0)) continue;
                int fj = face_of(L, j);
                if (fi == 1 && fj == 0) qi += gij * (1.0 - P[j]);
                if (fi == 0 && fj == 2) qo += gij * P[i];
                if (fi == 1 && fj == 2) { qi += gij; qo += gij; }
            }
    }
    *Qin = qi;
    *Qout = qo;
}

static double cross_section(const lat_t *L)
{
    double s = 1.0;
    for (int k = 0; k < L->dim; ++k)
        if (k != L->axis) s *= (double)L->n[k];
    return s;
}

/* ---------------------------------------------------------------- the solve */
/*
 * Preconditioned CG on the live set. The preconditioner M is diag(d) (Jacobi,
 * precond = 0) or the identity (precond = 1); the initial guess x_0 is the
 * linear profile 1 - c_axis / (n_axis - 1) on live nodes (x0 = 0, the exact
 * solution of a uniform network) or 0 (x0 = 1):
 *   r = b - A x_0, z = M^-1 r, p = z, rho = r.z
 *   repeat: q = A p; alpha = rho / p.q; x += alpha p; r -= alpha q;
 *           if ||r|| <= tol ||b||: recompute r = b - A x; stop if still below,
 *             otherwise continue from it with beta = 0, or stop (not
 *             converged) once that true residual fails to halve between checks;
 *           z = D^-1 r; rho' = r.z; beta = rho'/rho; p = z + beta p.
 * Then the energy form of the conductance, G = Q_in - x.(b - A x), which
 * equals sum over bonds g (dP)^2 and whose error is quadratic in the solution
 * error, and K from Eq. 4.
 */
int rno_solve(int dim, int64_t nx, int64_t ny, int64_t nz, int axis, int periodic,
              const double *g0, const double *g1, const double *g2,
              double tol, int64_t max_iter, int x0, int precond,
              double *p_out, uint8_t *mask_out, rno_result *res)
{
    lat_t L;
    int st = setup(&L, dim, nx, ny, nz, axis, periodic, g0, g1, g2);
    if (st) return st;
    if (!(tol > 0.0) || max_iter < 0 || !res) return RNO_EINVAL;
    if ((x0 != 0 && x0 != 1) || (precond != 0 && precond != 1)) return RNO_EINVAL;
    memset(res, 0, sizeof(*res));
    size_t N = (size_t)L.N;
    uint8_t *mask = (uint8_t *)malloc(N);
    double *d = (double *)malloc(N * sizeof(double));
    double *b = (double *)malloc(N * sizeof(double));
    double *x = (double *)calloc(N, sizeof(double));
    double *r = (double *)malloc(N * sizeof(double));
    double *z = (double *)malloc(N * sizeof(double));
    double *p = (double *)malloc(N * sizeof(double));
    double *q = (double *)malloc(N * sizeof(double));
    double *P = (double *)malloc(N * sizeof(double));
    if (!mask || !d || !b || !x || !r || !z || !p || !q || !P) { st = RNO_ENOMEM; goto done; }

    int64_t n_live = 0;
    st = mask_bfs(&L, mask, &n_live);
    if (st) goto done;
    assemble(&L, mask, d, b);

    double bnorm = sqrt(pdot(b, b, L.N));
    int64_t it = 0;
    int converged = 0;
    double rnorm = bnorm;
    if (n_live == 0 || bnorm == 0.0) {
        converged = 1;
        rnorm = 0.0;
    } else {
        if (x0 == 0) {
            const double span = (double)(L.n[L.axis] - 1);
            for (int64_t i = 0; i < L.N; ++i)
                x[i] = mask[i] == 3 ? 1.0 - (double)coord(&L, i, L.axis) / span : 0.0;
        }
        apply_A(&L, mask, d, x, q);
        for (size_t i = 0; i < N; ++i) r[i] = b[i] - q[i];
        for (size_t i = 0; i < N; ++i) {
            z[i] = mask[i] == 3 ? (precond == 0 ? r[i] / d[i] : r[i]) : 0.0;
            p[i] = z[i];
        }
        rnorm = sqrt(pdot(r, r, L.N));
        double rho = pdot(r, z, L.N);
        double last_check = INFINITY; /* true residual at the previous failed check */
        int restart = 0;
        if (rnorm <= tol * bnorm) converged = 1;   /* the initial guess already solves it */
        while (!converged && it < max_iter) {
            apply_A(&L, mask, d, p, q);
            double pq = pdot(p, q, L.N);
            if (!(pq > 0.0) || !isfinite(pq)) { st = RNO_ENUMERIC; break; }
            double alpha = rho / pq;
            for (size_t i = 0; i < N; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
            ++it;
            rnorm = sqrt(pdot(r, r, L.N));
            if (rnorm <= tol * bnorm) {
                apply_A(&L, mask, d, x, q);
                for (size_t i = 0; i < N; ++i) r[i] = b[i] - q[i];
                rnorm = sqrt(pdot(r, r, L.N));
                if (rnorm <= tol * bnorm) { converged = 1; break; }
                /* Not converged: carry on from the true residual with a fresh
                 * search direction; stop when the true residual no longer
                 * halves between checks (rounding floor reached). */
                if (!(rnorm < 0.5 * last_check)) break;
                last_check = rnorm;
                restart = 1;
            }
            for (size_t i = 0; i < N; ++i) z[i] = mask[i] == 3 ? (precond == 0 ? r[i] / d[i] : r[i]) : 0.0;
            double rho_new = pdot(r, z, L.N);
            double beta = restart ? 0.0 : rho_new / rho;
            restart = 0;
            rho = rho_new;
            for (size_t i = 0; i < N; ++i) p[i] = z[i] + beta * p[i];
        }
    }

    /* true residual of the final iterate, pressures, fluxes, energy, K */
    apply_A(&L, mask, d, x, q);
    for (size_t i = 0; i < N; ++i) r[i] = b[i] - q[i];
    rnorm = sqrt(pdot(r, r, L.N));
    fill_pressure(&L, mask, x, P);
    double Qin, Qout;
    face_fluxes(&L, P, &Qin, &Qout);
    double G = Qin - pdot(x, r, L.N);
    res->Q_in = Qin;
    res->Q_out = Qout;
    res->G = G;
    res->K = G * (double)(L.n[L.axis] - 1) / cross_section(&L);
    res->rel_resid = bnorm > 0.0 ? rnorm / bnorm : 0.0;
    res->iters = it;
    res->n_live = n_live;
    res->converged = converged;
    if (!st && !converged) st = RNO_ENOCONV;
    res->status = st;
    if (p_out) memcpy(p_out, P, N * sizeof(double));
    if (mask_out) memcpy(mask_out, mask, N);

done:
    free(mask); free(d); free(b); free(x); free(r); free(z); free(p); free(q); free(P);
    return st;
}

/* ------------------------------------------------ checks of a given pressure field */
/*
 * Given a full pressure field P (any source), evaluate with this file's own
 * mask and operator: the residual b - A x on the live set (x = P there), its
 * 2-norm, ||b||, the fluxes Q_in / Q_out of P, the energy conductance
 * G_E = Q_in - x.(b - A x), the minimum and maximum of P over live nodes, and
 * sum_i (A x - b)_i. out[] receives, in order:
 *   0 ||b - A x||, 1 ||b||, 2 Q_in, 3 Q_out, 4 G_E, 5 K_E, 6 min P_live,
 *   7 max P_live, 8 sum (A x - b), 9 n_live.
 */
int rno_check_pressure(int dim, int64_t nx, int64_t ny, int64_t nz, int axis, int periodic,
                       const double *g0, const double *g1, const double *g2,
                       const double *P_in, double *out)
{
    lat_t L;
    int st = setup(&L, dim, nx, ny, nz, axis, periodic, g0, g1, g2);
    if (st) return st;
    size_t N = (size_t)L.N;
    uint8_t *mask = (uint8_t *)malloc(N);
    double *d = (double *)malloc(N * sizeof(double));
    double *b = (double *)malloc(N * sizeof(double));
    double *x = (double *)malloc(N * sizeof(double));
    double *r = (double *)malloc(N * sizeof(double));
    double *P = (double *)malloc(N * sizeof(double));
    if (!mask || !d || !b || !x || !r || !P) { st = RNO_ENOMEM; goto done; }
    int64_t n_live = 0;
    st = mask_bfs(&L, mask, &n_live);
    if (st) goto done;
    assemble(&L, mask, d, b);
    double pmin = INFINITY, pmax = -INFINITY;
    for (size_t i = 0; i < N; ++i) {
        x[i] = mask[i] == 3 ? P_in[i] : 0.0;
        if (mask[i] == 3) {
            if (P_in[i] < pmin) pmin = P_in[i];
            if (P_in[i] > pmax) pmax = P_in[i];
        }
    }
    apply_A(&L, mask, d, x, r);
    double sum_res = 0.0;
    for (size_t i = 0; i < N; ++i) { sum_res += r[i] - b[i]; r[i] = b[i] - r[i]; }
    fill_pressure(&L, mask, x, P);
    double Qin, Qout;
    face_fluxes(&L, P, &Qin, &Qout);
    double G = Qin - pdot(x, r, L.N);
    out[0] = sqrt(pdot(r, r, L.N));
    out[1] = sqrt(pdot(b, b, L.N));
    out[2] = Qin;
    out[3] = Qout;
    out[4] = G;
    out[5] = G * (double)(L.n[L.axis] - 1) / cross_section(&L);
    out[6] = n_live ? pmin : 0.0;
    out[7] = n_live ? pmax : 0.0;
    out[8] = sum_res;
    out[9] = (double)n_live;
done:
    free(mask); free(d); free(b); free(x); free(r); free(P);
    return st;
}

/* ----------------------------------------------------------------- backbone */
/*
 * Backbone of the sample-spanning cluster. Near the percolation threshold the
 * spanning cluster grows tortuous (Sec. VI, the RRN study with q -> q_c = 1/2)
 * and most of its nodes sit on dangling ends: branches and loops that touch the
 * rest of the cluster through one node only and so carry no flow. The paper
 * does not define the backbone; this is the textbook definition: an interior
 * node is on the backbone when some path from an inlet-face node to an
 * outlet-face node passes through it without visiting any node twice.
 *
 * Equivalent form used here: contract the inlet face to one vertex S and the
 * outlet face to one vertex T (their nodes share one pressure each), keep the
 * live interior nodes and their occupied bonds (a bond from a live node to a
 * face node becomes an edge to S or T), and add one edge S-T. A node lies on a
 * simple S-T path exactly when it shares a biconnected component (block) with
 * that extra edge. The blocks come from Hopcroft and Tarjan's depth-first
 * search with a stack of edges (written iteratively, one frame per vertex):
 * when the search returns from v to its parent u with low(v) >= disc(u), the
 * edges above v's mark on the stack form one block.
 *
 * Edges are identified by the bond's storage slot (k * N + index of the entry
 * g[k][.] that holds it), so the two bonds between the same pair of nodes on a
 * periodic direction of extent 2 stay two edges; the S-T edge is 3 N.
 *
 * Output: the mask of mask_bfs with bit3 (8) set on every backbone node
 * (backbone nodes are 11, other live nodes 3); *n_backbone counts them.
 * Pinned by the tests against a brute-force vertex-cut check (Menger's theorem
 * on tiny networks), a hand-built network with a dangling loop, and the
 * physics: with an exact solve no bond of a live node off the backbone carries
 * current, and removing those nodes leaves K unchanged.
 */
typedef struct {
    const lat_t *L;
    const uint8_t *mask;
    int64_t S, T;
    const int64_t *adjS, *adjT;  /* nodes joined to S / T, each with its bond id */
    const int64_t *eidS, *eidT;
    int64_t nS, nT;
} bbg_t;

/* The pos-th incident edge of vertex v: returns 0 when pos is past the end,
 * -1 when that slot holds no edge, 1 with *w and *eid set otherwise. */
static int bb_edge(const bbg_t *G, int64_t v, int64_t pos, int64_t *w, int64_t *eid)
{
    const lat_t *L = G->L;
    if (v == G->S || v == G->T) {
        const int64_t cnt = v == G->S ? G->nS : G->nT;
        if (pos > cnt) return 0;
        if (pos == 0) { *w = v == G->S ? G->T : G->S; *eid = 3 * L->N; return 1; }
        *w = (v == G->S ? G->adjS : G->adjT)[pos - 1];
        *eid = (v == G->S ? G->eidS : G->eidT)[pos - 1];
        return 1;
    }
    if (pos >= 2 * L->dim) return 0;
    const int k = (int)(pos / 2), s = (pos & 1) ? 1 : -1;
    double gij;
    const int64_t j = nbr(L, v, k, s, &gij);
    if (j < 0 || !(gij > 0.0)) return -1;
    const int f = face_of(L, j);
    if (f == 1) *w = G->S;
    else if (f == 2) *w = G->T;
    else if (G->mask[j] == 3) *w = j;
    else return -1;
    *eid = (int64_t)k * L->N + (s > 0 ? v : j);
    return 1;
}

static int backbone(const lat_t *L, uint8_t *mask, int64_t *n_live, int64_t *n_backbone)
{
    int st = mask_bfs(L, mask, n_live);
    if (st) return st;
    const int64_t N = L->N, V = N + 2, S = N, T = N + 1;
    const int ax = L->axis;
    int64_t nS = 0, nT = 0;
    for (int64_t i = 0; i < N; ++i) {
        if (mask[i] != 3) continue;
        double gij;
        int64_t j = nbr(L, i, ax, -1, &gij);
        if (j >= 0 && gij > 0.0 && face_of(L, j) == 1) ++nS;
        j = nbr(L, i, ax, +1, &gij);
        if (j >= 0 && gij > 0.0 && face_of(L, j) == 2) ++nT;
    }
    int64_t *adjS = malloc(sizeof(int64_t) * (size_t)(nS + 1)), *eidS = malloc(sizeof(int64_t) * (size_t)(nS + 1));
    int64_t *adjT = malloc(sizeof(int64_t) * (size_t)(nT + 1)), *eidT = malloc(sizeof(int64_t) * (size_t)(nT + 1));
    int64_t *disc = malloc(sizeof(int64_t) * (size_t)V), *low = malloc(sizeof(int64_t) * (size_t)V);
    int64_t *peid = malloc(sizeof(int64_t) * (size_t)V), *pos = malloc(sizeof(int64_t) * (size_t)V);
    int64_t *mark = malloc(sizeof(int64_t) * (size_t)V), *vstk = malloc(sizeof(int64_t) * (size_t)V);
    const int64_t E = (int64_t)L->dim * N + 1;            /* at most one edge per bond slot, plus S-T */
    int64_t *ea = malloc(sizeof(int64_t) * (size_t)E), *eb = malloc(sizeof(int64_t) * (size_t)E);
    uint8_t *on = calloc((size_t)V, 1);
    int ok = adjS && eidS && adjT && eidT && disc && low && peid && pos && mark && vstk && ea && eb && on;
    if (ok) {
        nS = nT = 0;
        for (int64_t i = 0; i < N; ++i) {
            if (mask[i] != 3) continue;
            double gij;
            int64_t j = nbr(L, i, ax, -1, &gij);
            if (j >= 0 && gij > 0.0 && face_of(L, j) == 1) { adjS[nS] = i; eidS[nS++] = (int64_t)ax * N + j; }
            j = nbr(L, i, ax, +1, &gij);
            if (j >= 0 && gij > 0.0 && face_of(L, j) == 2) { adjT[nT] = i; eidT[nT++] = (int64_t)ax * N + i; }
        }
        const bbg_t G = {L, mask, S, T, adjS, adjT, eidS, eidT, nS, nT};
        for (int64_t v = 0; v < V; ++v) disc[v] = -1;
        int64_t clock = 0, top = 0, ne = 0;
        disc[S] = low[S] = clock++;
        peid[S] = -1;
        pos[S] = 0;
        vstk[top++] = S;
        while (top > 0) {
            const int64_t v = vstk[top - 1];
            int64_t w, eid;
            const int r = bb_edge(&G, v, pos[v], &w, &eid);
            if (r != 0) {
                ++pos[v];
                if (r < 0 || eid == peid[v]) continue;
                if (disc[w] < 0) {                       /* tree edge: descend */
                    mark[w] = ne;
                    ea[ne] = v; eb[ne++] = w;
                    disc[w] = low[w] = clock++;
                    peid[w] = eid;
                    pos[w] = 0;
                    vstk[top++] = w;
                } else if (disc[w] < disc[v]) {          /* back edge to an ancestor */
                    ea[ne] = v; eb[ne++] = w;
                    if (disc[w] < low[v]) low[v] = disc[w];
                }                                        /* else: seen from the other end already */
                continue;
            }
            --top;                                       /* v is finished */
            if (top == 0) break;
            const int64_t u = vstk[top - 1];
            if (low[v] < low[u]) low[u] = low[v];
            if (low[v] >= disc[u]) {                     /* the edges above mark[v] form a block */
                int st_edge = 0;
                for (int64_t e = mark[v]; e < ne; ++e)
                    if ((ea[e] == S && eb[e] == T) || (ea[e] == T && eb[e] == S)) st_edge = 1;
                if (st_edge)
                    for (int64_t e = mark[v]; e < ne; ++e) on[ea[e]] = on[eb[e]] = 1;
                ne = mark[v];
            }
        }
        int64_t nb = 0;
        for (int64_t i = 0; i < N; ++i)
            if (on[i] && mask[i] == 3) { mask[i] |= 8u; ++nb; }
        if (n_backbone) *n_backbone = nb;
    }
    free(adjS); free(eidS); free(adjT); free(eidT); free(disc); free(low); free(peid); free(pos);
    free(mark); free(vstk); free(ea); free(eb); free(on);
    return ok ? RNO_OK : RNO_ENOMEM;
}

int rno_backbone(int dim, int64_t nx, int64_t ny, int64_t nz, int axis, int periodic,
                 const double *g0, const double *g1, const double *g2,
                 uint8_t *mask_out, int64_t *n_live_out, int64_t *n_backbone_out)
{
    lat_t L;
    int st = setup(&L, dim, nx, ny, nz, axis, periodic, g0, g1, g2);
    if (st) return st;
    return backbone(&L, mask_out, n_live_out, n_backbone_out);
}
