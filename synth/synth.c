/*
 * Seeded synthetic inputs for the sparse CG path.
 *
 * This module produces the matrices and vectors that both the GPU library and
 * the CPU oracle consume.  It holds none of the solver's arithmetic (no SpMV,
 * no dot, no CG): only random streams, finite-difference / finite-element
 * stiffness assembly and right-hand-side sampling.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014).  uniform01 takes the top 53
 * bits; a standard normal is one Box-Muller draw (cosine branch) from two
 * consecutive uniforms.
 *
 * Matrices (CSR, 0-based int32 row starts / column indices, float64 values,
 * columns ascending inside every row, no duplicates):
 *   fd7      7-point finite-difference Laplacian on an N^3 interior grid,
 *            homogeneous Dirichlet boundary eliminated, integer stencil
 *            (6 on the diagonal, -1 per interior neighbour).
 *   q1cube   trilinear (Q1) hexahedral finite-element stiffness of
 *            -div(k grad u) on the unit cube, N^3 interior nodes on (N+1)^3
 *            elements, per-element coefficient k_e = exp(sigma * Z_e).  All 27
 *            structural neighbours are stored, the exact zeros on the 6 axis
 *            neighbours included, so nnz = (3N-2)^3.
 *   q1box    Q1 stiffness of the constant-coefficient Poisson problem on the
 *            200 x 200 x 10 km box of the paper's gravity model (Section 5.1),
 *            a x a x c nodes, boundary nodes kept as identity rows and their
 *            columns removed from interior rows.
 * Node numbering is lexicographic: i + Nx*(j + Ny*k).
 */
#define _USE_MATH_DEFINES
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- RNG -- */

static inline uint64_t sm64_next(uint64_t *s)
{
    uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline double sm64_u01(uint64_t *s)
{
    return (double)(sm64_next(s) >> 11) * 0x1.0p-53;
}

static inline double sm64_normal(uint64_t *s)
{
    double u1 = 1.0 - sm64_u01(s); /* (0, 1] so the log is finite */
    double u2 = sm64_u01(s);
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

/* Raw 64-bit outputs, for pinning the generator against its definition. */
void synth_splitmix64(uint64_t seed, int64_t n, uint64_t *out)
{
    uint64_t s = seed;
    for (int64_t i = 0; i < n; ++i) out[i] = sm64_next(&s);
}

/* out[i] = lo + (hi - lo) * u_i, u_i uniform on [0, 1). */
void synth_uniform(uint64_t seed, int64_t n, double lo, double hi, double *out)
{
    uint64_t s = seed;
    double w = hi - lo;
    for (int64_t i = 0; i < n; ++i) out[i] = lo + w * sm64_u01(&s);
}

void synth_normal(uint64_t seed, int64_t n, double *out)
{
    uint64_t s = seed;
    for (int64_t i = 0; i < n; ++i) out[i] = sm64_normal(&s);
}

/* ---------------------------------------------------------------- FD7 -- */

int64_t synth_fd7_nnz(int N)
{
    int64_t n = (int64_t)N * N * N;
    return n + 6 * (int64_t)N * N * (N - 1);
}

void synth_fd7(int N, int32_t *row_ptr, int32_t *col_idx, double *val)
{
    int64_t k = 0, row = 0;
    row_ptr[0] = 0;
    for (int z = 0; z < N; ++z)
        for (int y = 0; y < N; ++y)
            for (int x = 0; x < N; ++x, ++row) {
                /* ascending column order: -z, -y, -x, centre, +x, +y, +z */
                if (z > 0) { col_idx[k] = (int32_t)(row - (int64_t)N * N); val[k++] = -1.0; }
                if (y > 0) { col_idx[k] = (int32_t)(row - N); val[k++] = -1.0; }
                if (x > 0) { col_idx[k] = (int32_t)(row - 1); val[k++] = -1.0; }
                col_idx[k] = (int32_t)row; val[k++] = 6.0;
                if (x < N - 1) { col_idx[k] = (int32_t)(row + 1); val[k++] = -1.0; }
                if (y < N - 1) { col_idx[k] = (int32_t)(row + N); val[k++] = -1.0; }
                if (z < N - 1) { col_idx[k] = (int32_t)(row + (int64_t)N * N); val[k++] = -1.0; }
                row_ptr[row + 1] = (int32_t)k;
            }
}

/* Variable-coefficient 7-point operator of -div(k grad u) on the N^3 grid
 * (cell-centred finite volumes, unit spacing): node coefficients k_i =
 * exp(sigma * Z_i) in lexicographic order; the coupling across a face is the
 * harmonic mean 2 k_i k_j / (k_i + k_j); a face on the Dirichlet boundary
 * couples to the boundary value with k_i.  Off-diagonal = -face, diagonal =
 * sum of the six faces (so the matrix is SPD).  sigma = 0 gives fd7. */
void synth_fd7_var(int N, double sigma, uint64_t seed, int32_t *row_ptr, int32_t *col_idx,
                   double *val)
{
    const int64_t n = (int64_t)N * N * N;
    double *k = (double *)malloc((size_t)n * sizeof(double));
    uint64_t s = seed;
    for (int64_t i = 0; i < n; ++i) k[i] = exp(sigma * sm64_normal(&s));
    int64_t e = 0, row = 0;
    row_ptr[0] = 0;
    const int64_t strides[3] = {1, N, (int64_t)N * N};
    for (int z = 0; z < N; ++z)
        for (int y = 0; y < N; ++y)
            for (int x = 0; x < N; ++x, ++row) {
                const int c[3] = {x, y, z};
                double diag = 0.0;
                double off[6];
                int64_t oc[6];
                int no = 0;
                /* faces in ascending column order: -z, -y, -x, +x, +y, +z */
                const int dims[6] = {2, 1, 0, 0, 1, 2};
                const int sgn[6] = {-1, -1, -1, 1, 1, 1};
                for (int f = 0; f < 6; ++f) {
                    const int d = dims[f];
                    const int cc = c[d] + sgn[f];
                    if (cc < 0 || cc >= N) {
                        diag += k[row];
                        continue;
                    }
                    const int64_t nb = row + sgn[f] * strides[d];
                    const double w = 2.0 * k[row] * k[nb] / (k[row] + k[nb]);
                    diag += w;
                    off[no] = -w;
                    oc[no++] = nb;
                }
                /* emit: the three lower neighbours, the diagonal, the upper ones */
                int o = 0;
                while (o < no && oc[o] < row) {
                    col_idx[e] = (int32_t)oc[o];
                    val[e++] = off[o];
                    ++o;
                }
                col_idx[e] = (int32_t)row;
                val[e++] = diag;
                for (; o < no; ++o) {
                    col_idx[e] = (int32_t)oc[o];
                    val[e++] = off[o];
                }
                row_ptr[row + 1] = (int32_t)e;
            }
    free(k);
}

/* ----------------------------------------------------------------- Q1 -- */

/* Per-element coefficients of q1cube: (N+1)^3 values exp(sigma * Z), element
 * (ex, ey, ez) at index ex + (N+1)*(ey + (N+1)*ez). */
void synth_q1_coeffs(int N, double sigma, uint64_t seed, double *k_e)
{
    uint64_t s = seed;
    int64_t ne = (int64_t)(N + 1) * (N + 1) * (N + 1);
    for (int64_t e = 0; e < ne; ++e) k_e[e] = exp(sigma * sm64_normal(&s));
}

int64_t synth_q1cube_nnz(int N)
{
    int64_t m = 3 * (int64_t)N - 2;
    return m * m * m;
}

/* Unit-cube Q1 stiffness between local vertices that differ in d coordinates
 * (d = 0..3): the Kronecker form S(x)M(x)M + M(x)S(x)M + M(x)M(x)S with
 * S = [[1,-1],[-1,1]], M = [[1/3,1/6],[1/6,1/3]] evaluates exactly to these
 * four numbers. */
static const double kQ1Ref[4] = {1.0 / 3.0, 0.0, -1.0 / 12.0, -1.0 / 12.0};

/* Assemble q1cube from given element coefficients.  Node (x,y,z), 1 <= x,y,z
 * <= N in grid terms, is unknown x-1 + N*(y-1 + N*(z-1)).  The entry between
 * a node and a neighbour sums, over the elements they share (taken in
 * lexicographic element order), k_e * h * Kref.  Exact zeros are stored. */
void synth_q1cube_from_coeffs(int N, const double *k_e, int32_t *row_ptr, int32_t *col_idx,
                              double *val)
{
    const double h = 1.0 / (double)(N + 1);
    const int64_t NE = N + 1;
    int64_t k = 0, row = 0;
    row_ptr[0] = 0;
    for (int z = 1; z <= N; ++z)
        for (int y = 1; y <= N; ++y)
            for (int x = 1; x <= N; ++x, ++row) {
                for (int dz = -1; dz <= 1; ++dz) {
                    int nz = z + dz;
                    if (nz < 1 || nz > N) continue;
                    for (int dy = -1; dy <= 1; ++dy) {
                        int ny = y + dy;
                        if (ny < 1 || ny > N) continue;
                        for (int dx = -1; dx <= 1; ++dx) {
                            int nx = x + dx;
                            if (nx < 1 || nx > N) continue;
                            int hd = (dx != 0) + (dy != 0) + (dz != 0);
                            /* shared elements: along an axis where the offset
                             * is 0 both elements [c-1, c] qualify, otherwise
                             * only the one between the two nodes */
                            int ez0 = dz == 0 ? z - 1 : (dz < 0 ? z - 1 : z);
                            int ez1 = dz == 0 ? z : ez0;
                            int ey0 = dy == 0 ? y - 1 : (dy < 0 ? y - 1 : y);
                            int ey1 = dy == 0 ? y : ey0;
                            int ex0 = dx == 0 ? x - 1 : (dx < 0 ? x - 1 : x);
                            int ex1 = dx == 0 ? x : ex0;
                            double ksum = 0.0;
                            for (int ez = ez0; ez <= ez1; ++ez)
                                for (int ey = ey0; ey <= ey1; ++ey)
                                    for (int ex = ex0; ex <= ex1; ++ex)
                                        ksum += k_e[ex + NE * (ey + NE * (int64_t)ez)];
                            col_idx[k] = (int32_t)((nx - 1) + (int64_t)N * ((ny - 1) + (int64_t)N * (nz - 1)));
                            val[k++] = ksum * h * kQ1Ref[hd];
                        }
                    }
                }
                row_ptr[row + 1] = (int32_t)k;
            }
}

int synth_q1cube(int N, double sigma, uint64_t seed, int32_t *row_ptr, int32_t *col_idx,
                 double *val)
{
    int64_t ne = (int64_t)(N + 1) * (N + 1) * (N + 1);
    double *k_e = (double *)malloc((size_t)ne * sizeof(double));
    if (!k_e) return -1;
    synth_q1_coeffs(N, sigma, seed, k_e);
    synth_q1cube_from_coeffs(N, k_e, row_ptr, col_idx, val);
    free(k_e);
    return 0;
}

/* -------------------------------------------------- paper-shape Q1 box -- */

int64_t synth_q1box_nnz(int a, int c)
{
    int64_t n = (int64_t)a * a * c;
    int64_t ni = (int64_t)(a - 2) * (a - 2) * (c - 2);
    int64_t ma = 3 * (int64_t)a - 8, mc = 3 * (int64_t)c - 8;
    return ma * ma * mc + (n - ni);
}

/* Constant-coefficient Q1 Laplacian on an a x a x c node grid spanning
 * Lx x Ly x Lz (the paper's 200 x 200 x 10 km box).  The element stiffness on
 * a brick of sides (hx, hy, hz) is
 *   (hy hz / hx) S(x)M(x)M + (hx hz / hy) M(x)S(x)M + (hx hy / hz) M(x)M(x)S
 * with S, M the 1D unit stiffness / mass matrices.  Dirichlet nodes are kept
 * as identity rows; interior rows drop their boundary columns. */
void synth_q1box(int a, int c, double Lx, double Ly, double Lz, int32_t *row_ptr,
                 int32_t *col_idx, double *val)
{
    const double hx = Lx / (a - 1), hy = Ly / (a - 1), hz = Lz / (c - 1);
    const double wx = hy * hz / hx, wy = hx * hz / hy, wz = hx * hy / hz;
    /* per-axis 1D factors: S is 1 on a shared coordinate, -1 otherwise; the
     * mass entry is 1/3 (shared) or 1/6 (different), summed over the 2 or 1
     * elements sharing the pair along that axis */
    int64_t k = 0, row = 0;
    row_ptr[0] = 0;
    for (int z = 0; z < c; ++z)
        for (int y = 0; y < a; ++y)
            for (int x = 0; x < a; ++x, ++row) {
                int bnd = (x == 0 || x == a - 1 || y == 0 || y == a - 1 || z == 0 || z == c - 1);
                if (bnd) {
                    col_idx[k] = (int32_t)row;
                    val[k++] = 1.0;
                    row_ptr[row + 1] = (int32_t)k;
                    continue;
                }
                for (int dz = -1; dz <= 1; ++dz) {
                    int nz = z + dz;
                    for (int dy = -1; dy <= 1; ++dy) {
                        int ny = y + dy;
                        for (int dx = -1; dx <= 1; ++dx) {
                            int nx = x + dx;
                            if (nx == 0 || nx == a - 1 || ny == 0 || ny == a - 1 || nz == 0 ||
                                nz == c - 1)
                                continue;
                            /* 1D pieces, already summed over the elements that
                             * contain both nodes along the axis */
                            double sx = dx == 0 ? 2.0 : -1.0, mx = dx == 0 ? 2.0 / 3.0 : 1.0 / 6.0;
                            double sy = dy == 0 ? 2.0 : -1.0, my = dy == 0 ? 2.0 / 3.0 : 1.0 / 6.0;
                            double sz = dz == 0 ? 2.0 : -1.0, mz = dz == 0 ? 2.0 / 3.0 : 1.0 / 6.0;
                            col_idx[k] = (int32_t)(nx + (int64_t)a * (ny + (int64_t)a * nz));
                            val[k++] = wx * sx * my * mz + wy * mx * sy * mz + wz * mx * my * sz;
                        }
                    }
                }
                row_ptr[row + 1] = (int32_t)k;
            }
}

/* ------------------------------------------------------ right-hand side -- */

/* Nodal load of a density anomaly made of `nblobs` Gaussian blobs on the
 * q1cube grid: b_i = h^3 * 4*pi * drho(x_i) (lumped mass, gravitational
 * constant set to 1), drho(x) = sum_m A_m exp(-|x - c_m|^2 / (2 s_m^2)),
 * c_m ~ U(0,1)^3, s_m ~ U[0.03, 0.15], A_m ~ U[-1, 1], drawn in that order
 * per blob. */
void synth_blob_rhs(int N, int nblobs, uint64_t seed, double *b)
{
    uint64_t s = seed;
    double cx[64], cy[64], cz[64], sw[64], amp[64];
    if (nblobs > 64) nblobs = 64;
    for (int m = 0; m < nblobs; ++m) {
        cx[m] = sm64_u01(&s);
        cy[m] = sm64_u01(&s);
        cz[m] = sm64_u01(&s);
        sw[m] = 0.03 + 0.12 * sm64_u01(&s);
        amp[m] = 2.0 * sm64_u01(&s) - 1.0;
    }
    const double h = 1.0 / (double)(N + 1);
    const double scale = h * h * h * 4.0 * M_PI;
    int64_t row = 0;
    for (int z = 1; z <= N; ++z)
        for (int y = 1; y <= N; ++y)
            for (int x = 1; x <= N; ++x, ++row) {
                double px = x * h, py = y * h, pz = z * h, rho = 0.0;
                for (int m = 0; m < nblobs; ++m) {
                    double d2 = (px - cx[m]) * (px - cx[m]) + (py - cy[m]) * (py - cy[m]) +
                                (pz - cz[m]) * (pz - cz[m]);
                    rho += amp[m] * exp(-d2 / (2.0 * sw[m] * sw[m]));
                }
                b[row] = scale * rho;
            }
}
