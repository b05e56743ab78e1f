/*
 * CPU oracle for the reverse ray walk -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, single-threaded C that states what the GPU path must compute.
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code with the GPU library.
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared -ffp-contract=off -fno-fast-math
 *        (no contraction, so "a*b + c" is two roundings unless fma() is
 *        written out; float arithmetic is IEEE binary32 on x86-64 SSE).
 *
 * What is computed (paper sec. 2.3, "Computing direction-dependent
 * integrals"): for a source point Q and a direction m, the discrete integral
 * I(Q, m) = sum_k f_k * r_k over the leaves k of the contribution grid that
 * the ray R(t) = Q + m t, t >= 0, crosses before it leaves the unit box, with
 * r_k the chord of the ray in leaf k from the slab method (sec. 2.3.2) and
 * f = rho (column density N).  The attenuation is exp(-kappa N) (eq. of the
 * simplified transfer equation, sec. 2.1).
 *
 * Walk (sec. 2.3.1: DDA stepping, Morton encoding of the advanced position,
 * array lookup of the leaf, extent rebuilt from key + level, advance to the
 * next boundary), with the readings taken where the paper is silent:
 *   - unit box, max depth D, finest cell h = 2^-D, integer probe p = floor(Q 2^D);
 *   - leaf lookup: the largest i with key[i] <= Morton(p) (leaves tile Morton order);
 *   - slab far planes of leaf i only; the near side of leaf k+1 is the exit
 *     face of leaf k, so t_in is the previous t_out (first t_in = 0);
 *   - axis a bounds the leaf iff 1/m_a is finite (m_a == 0: ray parallel);
 *   - t_out = min of the far-plane times in the order x, y, z (strict <);
 *   - chord l = t_out - t_in, clamped at 0 (clamps are counted);
 *   - every bounding axis whose far time equals t_out is stepped to the
 *     neighbouring cell at once (edges and corners); the other axes take
 *     floor(fma(m_a, t_out, Q_a) 2^D) clamped to the current leaf;
 *   - the walk ends when the probe leaves [0, 2^D)^3.
 *
 * Directions: HEALPix RING pixel centres (Gorski et al. 2005, as used in
 * sec. 2.1), written here from the ring geometry.
 *
 * Several fields per leaf (orc_shielding): the same walk integrates every
 * field; the per-ray columns give the line optical depths and the per-source
 * escape probabilities of sec. 2.4 and the effective visual extinction of
 * sec. 3.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_ARG (-1)
#define ORC_ERR_UNSORTED (-2)
#define ORC_ERR_TILING (-3)
#define ORC_ERR_RANGE (-4)
#define ORC_ERR_STEPS (-7)

/* ------------------------------------------------------------------ */
/* HEALPix RING pixel centres                                          */
/* ------------------------------------------------------------------ */

int64_t orc_healpix_npix(int nside)
{
    if (nside < 1 || nside > (1 << 20)) return -1;
    return 12 * (int64_t)nside * (int64_t)nside;
}

/* dirs: [12 nside^2][3] unit vectors, ring by ring from the north pole,
 * azimuth ascending inside each ring. */
int orc_healpix_ring(int nside, double *dirs)
{
    if (orc_healpix_npix(nside) < 0 || !dirs) return ORC_ERR_ARG;
    const double pi = 3.14159265358979323846;
    const double ns = (double)nside;
    int64_t pix = 0;
    for (int64_t i = 1; i <= 4 * (int64_t)nside - 1; ++i) {
        double z;
        int64_t npr;          /* pixels in this ring */
        double dphi, phi0;    /* phi_j = phi0 + j * dphi, j = 0 .. npr-1 */
        if (i < nside) {                     /* north polar cap */
            z = 1.0 - (double)(i * i) / (3.0 * ns * ns);
            npr = 4 * i;
            dphi = pi / (2.0 * (double)i);
            phi0 = 0.5 * dphi;
        } else if (i <= 3 * (int64_t)nside) { /* equatorial belt */
            z = 4.0 / 3.0 - 2.0 * (double)i / (3.0 * ns);
            npr = 4 * (int64_t)nside;
            dphi = pi / (2.0 * ns);
            /* rings with (i - nside) even are shifted by half a pixel */
            phi0 = ((i - nside) % 2 == 0) ? 0.5 * dphi : 0.0;
        } else {                             /* south polar cap */
            int64_t ip = 4 * (int64_t)nside - i;
            z = -(1.0 - (double)(ip * ip) / (3.0 * ns * ns));
            npr = 4 * ip;
            dphi = pi / (2.0 * (double)ip);
            phi0 = 0.5 * dphi;
        }
        double st = sqrt((1.0 - z) * (1.0 + z));
        for (int64_t j = 0; j < npr; ++j) {
            double phi = phi0 + (double)j * dphi;
            dirs[3 * pix + 0] = st * cos(phi);
            dirs[3 * pix + 1] = st * sin(phi);
            dirs[3 * pix + 2] = z;
            ++pix;
        }
    }
    return ORC_OK;
}

/* NESTED order (Gorski et al. 2005), through the continuous HEALPix
 * projection of the sphere onto the plane (the projection that defines the
 * pixelisation; in its equatorial zone the plane coordinates are phi and
 * 3 pi z / 8, in its polar zones a point at sigma = sqrt(3 (1 - |z|)) keeps
 * its distance from the polar tooth's centre meridian scaled by sigma).
 * Here the plane is measured in units of pi/4: X = 4 phi / pi, Y = 4 y / pi.
 * Every base pixel is then a square of diagonal 2 turned by 45 degrees,
 * centred where the nside = 1 RING centres lie (z = 2/3, 0, -2/3 give
 * Y = 1, 0, -1; phi = pi/4 + k pi/2 or k pi/2 gives X = 1 + 2k or 2k):
 *   faces 0..3  (north)   centre (1 + 2f, 1),
 *   faces 4..7  (equator) centre (2 (f - 4), 0),
 *   faces 8..11 (south)   centre (1 + 2 (f - 8), -1).
 * Pixel p = f nside^2 + i: the even bits of i give its x and the odd bits
 * its y coordinate on the face; x runs from the face's south corner toward
 * its east corner, y toward its west corner, so the centre of (x, y) is
 *   X = Xc + (x - y) / nside,  Y = Yc - 1 + (x + y + 1) / nside.
 * Back onto the sphere: |Y| <= 1 (equatorial zone) gives z = 2 Y / 3 and
 * phi = pi X / 4; |Y| > 1 (polar zone) gives sigma = 2 - |Y|,
 * z = sign(Y) (1 - sigma^2 / 3) and phi = (pi / 4) (Xc + (X - Xc) / sigma),
 * Xc being the tooth's centre meridian, which is the face's own for a polar
 * face (the polar part of a north or south face lies inside its tooth). */
int orc_healpix_nested(int nside, double *dirs)
{
    int64_t npix = orc_healpix_npix(nside);
    if (npix < 0 || !dirs || (nside & (nside - 1))) return ORC_ERR_ARG;
    const double pi = 3.14159265358979323846;
    const double ns = (double)nside;
    const int64_t per_face = (int64_t)nside * (int64_t)nside;
    for (int64_t p = 0; p < npix; ++p) {
        int f = (int)(p / per_face);
        int64_t in_face = p % per_face, x = 0, y = 0;
        for (int b = 0; b < 32; ++b) {
            x |= ((in_face >> (2 * b)) & 1) << b;
            y |= ((in_face >> (2 * b + 1)) & 1) << b;
        }
        double Xc, Yc;
        if (f < 4) {
            Xc = 1.0 + 2.0 * f;
            Yc = 1.0;
        } else if (f < 8) {
            Xc = 2.0 * (f - 4);
            Yc = 0.0;
        } else {
            Xc = 1.0 + 2.0 * (f - 8);
            Yc = -1.0;
        }
        /* exact: dyadic fractions of a power-of-two nside */
        const double X = Xc + (double)(x - y) / ns;
        const double Y = Yc - 1.0 + (double)(x + y + 1) / ns;
        double z, phi;
        if (fabs(Y) <= 1.0) {
            z = 2.0 * Y / 3.0;
            phi = pi * X / 4.0;
        } else {
            const double sigma = 2.0 - fabs(Y);
            z = (1.0 - sigma * sigma / 3.0) * (Y > 0.0 ? 1.0 : -1.0);
            phi = pi * (Xc + (X - Xc) / sigma) / 4.0;
        }
        const double st = sqrt((1.0 - z) * (1.0 + z));
        dirs[3 * p + 0] = st * cos(phi);
        dirs[3 * p + 1] = st * sin(phi);
        dirs[3 * p + 2] = z;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Linear octree: Morton keys, tiling check, leaf lookup               */
/* ------------------------------------------------------------------ */

/* Morton key of the integer point (x, y, z) at depth D: bit b of x goes to
 * bit 3b, of y to 3b+1, of z to 3b+2. */
static uint64_t morton_key(int64_t x, int64_t y, int64_t z, int depth)
{
    uint64_t k = 0;
    for (int b = 0; b < depth; ++b) {
        k |= (uint64_t)((x >> b) & 1) << (3 * b);
        k |= (uint64_t)((y >> b) & 1) << (3 * b + 1);
        k |= (uint64_t)((z >> b) & 1) << (3 * b + 2);
    }
    return k;
}

uint64_t orc_morton(int64_t x, int64_t y, int64_t z, int depth)
{
    return morton_key(x, y, z, depth);
}

/* Leaves must be sorted, aligned to their own size, and tile [0, 8^D). */
int orc_check_tiling(const uint64_t *keys, const uint8_t *levels, int64_t n, int depth)
{
    if (!keys || !levels || n < 1 || depth < 1 || depth > 21) return ORC_ERR_ARG;
    for (int64_t i = 1; i < n; ++i)
        if (keys[i] <= keys[i - 1]) return ORC_ERR_UNSORTED;
    uint64_t expect = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (levels[i] > depth) return ORC_ERR_TILING;
        uint64_t span = (uint64_t)1 << (3 * (depth - levels[i]));
        if (keys[i] % span != 0) return ORC_ERR_TILING;
        if (keys[i] != expect) return ORC_ERR_TILING;
        expect = keys[i] + span;
    }
    if (expect != (uint64_t)1 << (3 * depth)) return ORC_ERR_TILING;
    return ORC_OK;
}

/* Largest i with keys[i] <= k (keys sorted, keys[0] == 0 <= k). */
static int64_t find_leaf(const uint64_t *keys, int64_t n, uint64_t k)
{
    int64_t lo = 0, hi = n; /* answer in [lo, hi) */
    while (hi - lo > 1) {
        int64_t mid = lo + (hi - lo) / 2;
        if (keys[mid] <= k) lo = mid; else hi = mid;
    }
    return lo;
}

/* ------------------------------------------------------------------ */
/* One ray                                                             */
/* ------------------------------------------------------------------ */

typedef struct {
    double N;          /* sum rho * l in FP64, visiting order, no fma */
    float N32;         /* sum rho32 * l32 in FP32 with Kahan compensation */
    double texit;      /* last t_out */
    int64_t steps;     /* leaves visited */
    uint64_t hash;     /* FNV-1a style hash of the visited leaf indices */
    int64_t clamps;    /* chords clamped at 0 */
} ray_out;

#define HASH0 0xcbf29ce484222325ULL
#define HASHP 0x100000001b3ULL

/* Walk one ray.  Visited leaf indices and chords go to vis/chords (first cap
 * entries; either may be NULL).  rho32 may be NULL (then N32 = 0). */
static int walk_ray(const uint64_t *keys, const uint8_t *levels, const double *rho,
                    const float *rho32, int64_t n, int depth, const double Q[3],
                    const double m[3], ray_out *o, int64_t *vis, double *chords, int64_t cap)
{
    const double scale = ldexp(1.0, depth);
    const double h = ldexp(1.0, -depth);
    const int64_t side = (int64_t)1 << depth;
    double inv[3];
    int bounding[3];
    int any = 0;
    memset(o, 0, sizeof(*o));
    o->hash = HASH0;
    for (int a = 0; a < 3; ++a) {
        if (!(Q[a] >= 0.0 && Q[a] < 1.0)) return ORC_ERR_RANGE;
        if (!isfinite(m[a])) return ORC_ERR_ARG;
        inv[a] = 1.0 / m[a];
        bounding[a] = isfinite(inv[a]);
        any |= bounding[a];
    }
    if (!any) return ORC_ERR_ARG;

    int64_t p[3];
    for (int a = 0; a < 3; ++a) p[a] = (int64_t)floor(Q[a] * scale);

    double t_in = 0.0, N = 0.0;
    float S = 0.0f, c = 0.0f;
    const int64_t max_steps = 3 * side + 3;
    for (int64_t step = 0;; ++step) {
        if (step >= max_steps) return ORC_ERR_STEPS;
        /* locate the leaf that holds the probe */
        uint64_t k = morton_key(p[0], p[1], p[2], depth);
        int64_t i = find_leaf(keys, n, k);
        int64_t size = (int64_t)1 << (depth - levels[i]);
        int64_t anchor[3];
        for (int a = 0; a < 3; ++a) anchor[a] = p[a] - p[a] % size;

        /* slab method: far-plane times of the leaf's box */
        double tf[3];
        for (int a = 0; a < 3; ++a) {
            if (bounding[a]) {
                int64_t plane = m[a] > 0.0 ? anchor[a] + size : anchor[a];
                tf[a] = ((double)plane * h - Q[a]) * inv[a];
            } else {
                tf[a] = INFINITY;
            }
        }
        double t_out = tf[0];
        if (tf[1] < t_out) t_out = tf[1];
        if (tf[2] < t_out) t_out = tf[2];

        /* path length in the leaf and its contribution */
        double l = t_out - t_in;
        if (l < 0.0) {
            l = 0.0;
            o->clamps += 1;
        } else {
            t_in = t_out;
        }
        N = N + rho[i] * l;
        if (rho32) {
            float y = rho32[i] * (float)l - c;
            float t = S + y;
            c = (t - S) - y;
            S = t;
        }
        if (vis && o->steps < cap) vis[o->steps] = i;
        if (chords && o->steps < cap) chords[o->steps] = l;
        o->hash = (o->hash ^ (uint64_t)i) * HASHP;
        o->steps += 1;

        /* advance to the next cell */
        int out = 0;
        for (int a = 0; a < 3; ++a) {
            if (bounding[a] && tf[a] == t_out) {
                p[a] = m[a] > 0.0 ? anchor[a] + size : anchor[a] - 1;
            } else {
                double x = fma(m[a], t_out, Q[a]) * scale;
                int64_t q = (int64_t)floor(x);
                if (q < anchor[a]) q = anchor[a];
                if (q > anchor[a] + size - 1) q = anchor[a] + size - 1;
                p[a] = q;
            }
            if (p[a] < 0 || p[a] >= side) out = 1;
        }
        if (out) break;
    }
    o->N = N;
    o->N32 = S;
    o->texit = t_in;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Exported entry points                                               */
/* ------------------------------------------------------------------ */

/* One ray, with its visited leaves and chords (first cap of them). */
int orc_walk_one(const uint64_t *keys, const uint8_t *levels, const double *rho,
                 const float *rho32, int64_t n, int depth, const double *Q, const double *m,
                 double *N, float *N32, double *texit, int64_t *steps, uint64_t *hash,
                 int64_t *clamps, int64_t *vis, double *chords, int64_t cap)
{
    ray_out o;
    int st = walk_ray(keys, levels, rho, rho32, n, depth, Q, m, &o, vis, chords, cap);
    if (N) *N = o.N;
    if (N32) *N32 = o.N32;
    if (texit) *texit = o.texit;
    if (steps) *steps = o.steps;
    if (hash) *hash = o.hash;
    if (clamps) *clamps = o.clamps;
    return st;
}

/* All rays (s, d) for S sources and Dn directions.  Outputs are [S][Dn]
 * row-major; any output pointer may be NULL.  A64 = exp(-kappa N) in FP64,
 * A32 = expf(-(float)kappa * N32).  Returns the first error, after filling
 * NaN into the failing ray's N. */
int orc_columns(const uint64_t *keys, const uint8_t *levels, const double *rho,
                const float *rho32, int64_t n, int depth, const double *src, int64_t S,
                const double *dirs, int64_t Dn, double kappa, double *N64, double *A64,
                float *N32, float *A32, double *texit, int64_t *steps, uint64_t *hash,
                int64_t *clamps_total)
{
    int status = ORC_OK;
    int64_t clamps = 0;
    for (int64_t s = 0; s < S; ++s) {
        for (int64_t d = 0; d < Dn; ++d) {
            ray_out o;
            int st = walk_ray(keys, levels, rho, rho32, n, depth, src + 3 * s, dirs + 3 * d, &o,
                              NULL, NULL, 0);
            int64_t r = s * Dn + d;
            if (st != ORC_OK) {
                if (status == ORC_OK) status = st;
                o.N = NAN;
                o.N32 = NAN;
                o.steps = -1;
            }
            clamps += o.clamps;
            if (N64) N64[r] = o.N;
            if (A64) A64[r] = exp(-kappa * o.N);
            if (N32) N32[r] = o.N32;
            if (A32) A32[r] = expf(-(float)kappa * o.N32);
            if (texit) texit[r] = o.texit;
            if (steps) steps[r] = o.steps;
            if (hash) hash[r] = o.hash;
        }
    }
    if (clamps_total) *clamps_total = clamps;
    return status;
}

/* Gradient of L with respect to the leaf values, given g = dL/dN per ray
 * ([S][Dn], FP64): since N(s,d) = sum_k rho_k l_k(s,d) with the chords fixed
 * by the topology, dL/drho_k = sum over rays of g * l_k.  grad is [n],
 * accumulated (+=). */
int orc_gradient(const uint64_t *keys, const uint8_t *levels, int64_t n, int depth,
                 const double *src, int64_t S, const double *dirs, int64_t Dn,
                 const double *g, double *grad)
{
    int64_t cap = 3 * ((int64_t)1 << depth) + 3;
    int64_t *vis = (int64_t *)malloc(sizeof(int64_t) * cap);
    double *chords = (double *)malloc(sizeof(double) * cap);
    double *zero = (double *)calloc((size_t)n, sizeof(double));
    if (!vis || !chords || !zero) {
        free(vis);
        free(chords);
        free(zero);
        return ORC_ERR_ARG;
    }
    int status = ORC_OK;
    for (int64_t s = 0; s < S && status == ORC_OK; ++s) {
        for (int64_t d = 0; d < Dn; ++d) {
            ray_out o;
            int st = walk_ray(keys, levels, zero, NULL, n, depth, src + 3 * s, dirs + 3 * d, &o,
                              vis, chords, cap);
            if (st != ORC_OK) {
                status = st;
                break;
            }
            double gr = g[s * Dn + d];
            for (int64_t j = 0; j < o.steps; ++j) grad[vis[j]] += gr * chords[j];
        }
    }
    free(vis);
    free(chords);
    free(zero);
    return status;
}

/* ------------------------------------------------------------------ */
/* Several fields per leaf: line optical depths, escape probabilities  */
/* and the effective visual extinction                                 */
/* ------------------------------------------------------------------ */

/* CGS constants (CODATA 2018): Boltzmann constant, proton mass, speed of light. */
#define ORC_KB 1.380649e-16
#define ORC_MP 1.67262192369e-24
#define ORC_C 2.99792458e10

/* Direction-dependent integrals of several leaf fields, and their
 * per-source reductions over directions (paper sec. 2.4 and sec. 3).
 *
 * fields is [n][K]: per leaf, field 0 is the hydrogen number density n_H and
 * field f = 1 .. K-1 is the level-population term [n_j g_i / g_j - n_i] of
 * line f, whose Einstein coefficient and frequency are lineA[f-1] and
 * linenu[f-1].  For the ray (s, d) of walk_ray (box units):
 *   I_f   = sum over visited leaves k of fields[k][f] * r_k, in visiting
 *           order, I = I + F r (the discrete integral of sec. 2.3);
 *   N_f   = length * I_f, the column in cm^-2 for a box edge of length cm;
 *   du    = sqrt(8 kB T_s / (pi m_p) + vturb^2), the rms of thermal and
 *           turbulent speed at the source (sec. 2.4);
 *   tau_f = coef_f * N_f / du with coef_f = A c^3 / (8 pi nu^3) (discretised
 *           line optical depth, sec. 2.4).
 * Per source, over its Dn directions d = 0 .. Dn-1:
 *   beta_f = (1/Dn) sum_d (1 - exp(-tau_f)) / tau_f, the escape probability
 *            (sec. 2.4); the term is its limit 1 at tau = 0 and is evaluated
 *            as -expm1(-tau) / tau otherwise, for every sign of tau;
 *   AV_eff = -(1/gamma) ln((1/Dn) sum_d exp(-gamma av0 N_H)) (sec. 3), evaluated
 *            with x_d = gamma av0 N_H,d and x_min = min_d x_d as
 *            (x_min - ln((1/Dn) sum_d exp(-(x_d - x_min)))) / gamma, which is
 *            the same number but does not underflow for large columns.
 * Outputs, each may be NULL: rays [S][Dn][K] with N_H at f = 0 and tau_f at
 * f >= 1; av_eff [S]; beta [S][K-1].  temp [S] (kelvin) is needed when
 * K > 1.  A source with an invalid ray, or with du not finite and > 0, gets
 * NaN in all its outputs, and the first such error is returned. */
int orc_shielding(const uint64_t *keys, const uint8_t *levels, int64_t n, int depth,
                  const double *fields, int K, const double *src, int64_t S,
                  const double *dirs, int64_t Dn, double length, const double *temp,
                  double vturb, const double *lineA, const double *linenu, double gamma,
                  double av0, double *rays, double *av_eff, double *beta)
{
    const double pi = 3.14159265358979323846;
    if (K < 1 || !fields || (K > 1 && (!temp || !lineA || !linenu)) || S < 0 || Dn < 1)
        return ORC_ERR_ARG;
    int64_t cap = 3 * ((int64_t)1 << depth) + 3;
    int64_t *vis = (int64_t *)malloc(sizeof(int64_t) * cap);
    double *chords = (double *)malloc(sizeof(double) * cap);
    double *zero = (double *)calloc((size_t)n, sizeof(double));
    double *I = (double *)malloc(sizeof(double) * K);
    double *coef = (double *)malloc(sizeof(double) * K);
    double *bsum = (double *)malloc(sizeof(double) * K);
    double *x = (double *)malloc(sizeof(double) * Dn);
    if (!vis || !chords || !zero || !I || !coef || !bsum || !x) {
        free(vis); free(chords); free(zero); free(I); free(coef); free(bsum); free(x);
        return ORC_ERR_ARG;
    }
    for (int f = 1; f < K; ++f) {
        const double nu = linenu[f - 1];
        coef[f] = lineA[f - 1] * (ORC_C * ORC_C * ORC_C) / (8.0 * pi * (nu * nu * nu));
    }
    int status = ORC_OK;
    for (int64_t s = 0; s < S; ++s) {
        int bad = 0;
        double du = 1.0;
        if (K > 1) {
            du = sqrt(8.0 * ORC_KB * temp[s] / (pi * ORC_MP) + vturb * vturb);
            if (!(du > 0.0 && isfinite(du))) {
                bad = 1;
                if (status == ORC_OK) status = ORC_ERR_RANGE;
            }
        }
        for (int f = 0; f < K; ++f) bsum[f] = 0.0;
        for (int64_t d = 0; d < Dn && !bad; ++d) {
            ray_out o;
            int st = walk_ray(keys, levels, zero, NULL, n, depth, src + 3 * s, dirs + 3 * d, &o,
                              vis, chords, cap);
            if (st != ORC_OK) {
                bad = 1;
                if (status == ORC_OK) status = st;
                break;
            }
            for (int f = 0; f < K; ++f) I[f] = 0.0;
            for (int64_t j = 0; j < o.steps; ++j)
                for (int f = 0; f < K; ++f) I[f] = I[f] + fields[vis[j] * K + f] * chords[j];
            const double nh = length * I[0];
            x[d] = gamma * av0 * nh;
            if (rays) rays[(s * Dn + d) * K] = nh;
            for (int f = 1; f < K; ++f) {
                const double tau = coef[f] * (length * I[f]) / du;
                bsum[f] += tau == 0.0 ? 1.0 : -expm1(-tau) / tau;
                if (rays) rays[(s * Dn + d) * K + f] = tau;
            }
        }
        if (bad) {
            if (rays)
                for (int64_t j = 0; j < Dn * K; ++j) rays[s * Dn * K + j] = NAN;
            if (av_eff) av_eff[s] = NAN;
            if (beta)
                for (int f = 1; f < K; ++f) beta[s * (K - 1) + f - 1] = NAN;
            continue;
        }
        double xmin = x[0];
        for (int64_t d = 1; d < Dn; ++d)
            if (x[d] < xmin) xmin = x[d];
        double sum = 0.0;
        for (int64_t d = 0; d < Dn; ++d) sum += exp(-(x[d] - xmin));
        if (av_eff) av_eff[s] = (xmin - log(sum / (double)Dn)) / gamma;
        if (beta)
            for (int f = 1; f < K; ++f) beta[s * (K - 1) + f - 1] = bsum[f] / (double)Dn;
    }
    free(vis); free(chords); free(zero); free(I); free(coef); free(bsum); free(x);
    return status;
}

/* ------------------------------------------------------------------ */
/* Angular-resolution comparison                                       */
/* ------------------------------------------------------------------ */

/* Reference columns of a coarse HEALPix NESTED direction set from a finer
 * one (sec. 3: the reference of a ray is the mean of the reference-resolution
 * rays inside its pixel; with ratio = Dfine / Dcoarse = 4^k these are the
 * fine rays q ratio .. (q+1) ratio - 1).  fine is [S][Dfine], coarse, ref and
 * err are [S][Dcoarse]; ref = (sum in index order) / ratio and
 * err = |coarse - ref| / ref.  coarse/err may be NULL together. */
int orc_nested_reference(const double *fine, int64_t Dfine, const double *coarse, int64_t Dcoarse,
                         int64_t S, double *ref, double *err)
{
    if (!fine || Dcoarse < 1 || S < 0 || Dfine % Dcoarse != 0) return ORC_ERR_ARG;
    const int64_t ratio = Dfine / Dcoarse;
    for (int64_t s = 0; s < S; ++s) {
        for (int64_t q = 0; q < Dcoarse; ++q) {
            double sum = 0.0;
            for (int64_t k = 0; k < ratio; ++k) sum = sum + fine[s * Dfine + q * ratio + k];
            const double r = sum / (double)ratio;
            if (ref) ref[s * Dcoarse + q] = r;
            if (err && coarse) err[s * Dcoarse + q] = fabs(coarse[s * Dcoarse + q] - r) / r;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Contribution grid from a uniform grid                               */
/* ------------------------------------------------------------------ */

/* The leaf-only octree of the paper's refinement rule (sec. 2.4, the AMR
 * contribution grid): starting from the root, a cell of level L < D is
 * split into its 8 children iff its largest fine value reaches floor and
 * its relative variation (max - min) / max reaches rel, evaluated as
 * max >= floor && (max - min) >= rel * max over the fine cells it covers;
 * an unsplit cell, or a cell at level D, is a leaf.  A leaf's value is the
 * mean of its fine cells, defined level by level as the mean of its 8
 * children's values (summed in child order, divided by 8).
 * grid is [8^D] in Morton order (fine cell i has key i).  Outputs, in
 * Morton order: keys, levels, values (capacity 8^D each); *n = leaf count. */

static int64_t tree_cells_before(int L) { return (((int64_t)1 << (3 * L)) - 1) / 7; }

static void emit_leaves(int L, int64_t c, int D, const double *mx, const double *mn,
                        const double *mean, const double *grid, double floor_, double rel,
                        uint64_t *keys, uint8_t *levels, double *values, int64_t *n)
{
    int split = 0;
    if (L < D) {
        const int64_t at = tree_cells_before(L) + c;
        split = mx[at] >= floor_ && (mx[at] - mn[at]) >= rel * mx[at];
    }
    if (!split) {
        keys[*n] = (uint64_t)c << (3 * (D - L));
        levels[*n] = (uint8_t)L;
        values[*n] = L < D ? mean[tree_cells_before(L) + c] : grid[c];
        *n += 1;
        return;
    }
    for (int j = 0; j < 8; ++j)
        emit_leaves(L + 1, 8 * c + j, D, mx, mn, mean, grid, floor_, rel, keys, levels, values, n);
}

int orc_grid_tree(const double *grid, int D, double floor_, double rel, uint64_t *keys,
                  uint8_t *levels, double *values, int64_t *n)
{
    if (!grid || D < 0 || D > 10 || !keys || !levels || !values || !n) return ORC_ERR_ARG;
    const int64_t cells = tree_cells_before(D);  /* all cells of levels 0 .. D-1 */
    double *mx = (double *)malloc(sizeof(double) * (cells > 0 ? cells : 1));
    double *mn = (double *)malloc(sizeof(double) * (cells > 0 ? cells : 1));
    double *mean = (double *)malloc(sizeof(double) * (cells > 0 ? cells : 1));
    if (!mx || !mn || !mean) {
        free(mx); free(mn); free(mean);
        return ORC_ERR_ARG;
    }
    /* max, min and mean of every cell, from level D-1 up to the root */
    for (int L = D - 1; L >= 0; --L) {
        const int64_t count = (int64_t)1 << (3 * L);
        for (int64_t c = 0; c < count; ++c) {
            double hi = -INFINITY, lo = INFINITY, sum = 0.0;
            for (int j = 0; j < 8; ++j) {
                const int64_t child = 8 * c + j;
                double chi, clo, cmean;
                if (L + 1 == D) {
                    chi = clo = cmean = grid[child];
                } else {
                    const int64_t at = tree_cells_before(L + 1) + child;
                    chi = mx[at];
                    clo = mn[at];
                    cmean = mean[at];
                }
                if (chi > hi) hi = chi;
                if (clo < lo) lo = clo;
                sum = sum + cmean;
            }
            const int64_t at = tree_cells_before(L) + c;
            mx[at] = hi;
            mn[at] = lo;
            mean[at] = sum / 8.0;
        }
    }
    *n = 0;
    emit_leaves(0, 0, D, mx, mn, mean, grid, floor_, rel, keys, levels, values, n);
    free(mx); free(mn); free(mean);
    return ORC_OK;
}
