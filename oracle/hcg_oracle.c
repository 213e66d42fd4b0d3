/*
 * hcg_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT PATH.
 *
 * A plain, slow, obviously-correct FP64 CPU oracle for single-dish
 * convolution-based gridding as defined by HCGrid (Wang et al. 2020, MNRAS):
 *
 *   - Eq. (1), Section 2.1: V[g] = (1/W_g) * sum_n V[s_n] w(g, n),
 *     W_g = sum_n w(g, n), with the Gaussian kernel of Section 3.6 (iii)
 *     truncated at the support radius ("sphere_radius").
 *   - The HEALPix ring-scheme pixelisation used for pre-ordering
 *     (Section 3.2; Gorski et al. 2005 give the geometry written out here).
 *
 * Only tests/, the smoke check and the benchmark's CPU-baseline leg may load
 * this library.  It shares no code, header or constant table with the HIP
 * path; the two meet only through the seeded input generators.
 *
 * Conventions (the paper is silent on these; the same readings are used on
 * every side):
 *   - angles enter in degrees; radians = degrees * 0.017453292519943295;
 *   - distance d is the great-circle distance (haversine form), a pair
 *     contributes iff d <= R (closed support);
 *   - w = exp(-d^2 / (2 sigma^2)), sigma = FWHM / (2 sqrt(2 ln 2)), peak 1;
 *   - a cell with no sample inside R has W = 0 and V = NaN;
 *   - grid cell (ix, iy) has centre lon0 + (ix - (nx-1)/2) dlon,
 *     lat0 + (iy - (ny-1)/2) dlat (a linear lon/lat grid);
 *   - every sum is a Neumaier-compensated FP64 sum.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_DEG2RAD 0.017453292519943295
#define ORC_PI 3.141592653589793

/* ------------------------------------------------------------------------ */
/* HEALPix ring scheme (Section 3.2; Gorski et al. 2005).                    */
/* Rings are numbered i = 1 .. 4*Ns-1 from the north pole.                   */
/* ------------------------------------------------------------------------ */

static int64_t floordiv_i64(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) q -= 1;
  return q;
}

static int64_t mod_i64(int64_t a, int64_t m) {
  int64_t r = a % m;
  return r < 0 ? r + m : r;
}

int64_t orc_hpx_npix(int64_t ns) { return 12 * ns * ns; }

/* number of pixels in ring i */
int64_t orc_hpx_ring_npix(int64_t ns, int64_t i) {
  if (i < 1 || i > 4 * ns - 1) return 0;
  if (i < ns) return 4 * i;
  if (i <= 3 * ns) return 4 * ns;
  return 4 * (4 * ns - i);
}

/* index of the first pixel of ring i */
int64_t orc_hpx_ring_start(int64_t ns, int64_t i) {
  if (i <= ns) return 2 * i * (i - 1);
  if (i <= 3 * ns) return 2 * ns * (ns - 1) + 4 * ns * (i - ns);
  int64_t s = 4 * ns - i; /* ring counted from the south pole */
  return 12 * ns * ns - 2 * s * (s + 1);
}

/* z = cos(colatitude) of the centres of ring i */
double orc_hpx_ring_z(int64_t ns, int64_t i) {
  double n = (double)ns;
  if (i < ns) return 1.0 - (double)(i * i) / (3.0 * n * n);
  if (i <= 3 * ns) return 4.0 / 3.0 - 2.0 * (double)i / (3.0 * n);
  int64_t s = 4 * ns - i;
  return -(1.0 - (double)(s * s) / (3.0 * n * n));
}

/* ring holding pixel p: the largest i with ring_start(i) <= p (bisection) */
int64_t orc_hpx_pix2ring(int64_t ns, int64_t p) {
  int64_t lo = 1, hi = 4 * ns - 1;
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) / 2;
    if (orc_hpx_ring_start(ns, mid) <= p) lo = mid; else hi = mid - 1;
  }
  return lo;
}

/* centre of pixel p, degrees (lon in [0, 360)) */
void orc_hpx_pix2ang(int64_t ns, int64_t p, double* lon_deg, double* lat_deg) {
  int64_t i = orc_hpx_pix2ring(ns, p);
  int64_t j = p - orc_hpx_ring_start(ns, i);
  double z = orc_hpx_ring_z(ns, i);
  double phi;
  if (i < ns || i > 3 * ns) {
    int64_t r = (i < ns) ? i : 4 * ns - i; /* ring number from the nearest pole */
    phi = (ORC_PI / (2.0 * (double)r)) * ((double)j + 0.5);
  } else {
    int64_t s = (i - ns + 1) % 2; /* belt rings alternate a half-pixel shift */
    phi = (ORC_PI / (2.0 * (double)ns)) * ((double)j + 0.5 * (double)s);
  }
  *lon_deg = phi / ORC_DEG2RAD;
  *lat_deg = asin(z) / ORC_DEG2RAD;
}

/*
 * Pixel containing (lon, lat).  t = 2 phi / pi in [0, 4), z = sin(lat).
 * Equatorial belt (|z| <= 2/3): pixel edges are the two families of lines
 *   Ns (1/2 + t - 3z/4) = integer  (ascending)   and
 *   Ns (1/2 + t + 3z/4) = integer  (descending),
 * so the pair of integer parts locates the pixel (its ring from their
 * difference, its position along the ring from their sum).
 * Polar caps (|z| > 2/3): with tau = t - floor(t) and q = Ns sqrt(3 (1-|z|)),
 * the edges are tau q = integer and (1 - tau) q = integer; the ring counted
 * from the pole is the sum of the two integer parts plus one, and the pixel
 * along that ring is floor(t * ring).
 */
int64_t orc_hpx_ang2pix(int64_t ns, double lon_deg, double lat_deg) {
  double lon = fmod(lon_deg, 360.0);
  if (lon < 0.0) lon += 360.0;
  if (lon >= 360.0) lon -= 360.0;
  double t = lon / 90.0;
  double z = sin(lat_deg * ORC_DEG2RAD);
  double za = fabs(z);
  double n = (double)ns;
  if (za <= 2.0 / 3.0) {
    double a = n * (0.5 + t);
    double b = n * z * 0.75;
    int64_t jp = (int64_t)floor(a - b); /* ascending-edge index  */
    int64_t jm = (int64_t)floor(a + b); /* descending-edge index */
    int64_t ir = ns + 1 + jp - jm;      /* 1 .. 2Ns+1, counted from z = 2/3 */
    int64_t odd = ir & 1;
    int64_t ip = floordiv_i64(jp + jm - ns + (1 - odd) + 1, 2);
    ip = mod_i64(ip, 4 * ns);
    return 2 * ns * (ns - 1) + (ir - 1) * 4 * ns + ip;
  }
  double tau = t - floor(t);
  double q = n * sqrt(3.0 * (1.0 - za));
  int64_t jp = (int64_t)floor(tau * q);
  int64_t jm = (int64_t)floor((1.0 - tau) * q);
  int64_t ir = jp + jm + 1; /* ring counted from the nearest pole */
  int64_t ip = (int64_t)floor(t * (double)ir);
  ip = mod_i64(ip, 4 * ir);
  if (z > 0.0) return 2 * ir * (ir - 1) + ip;
  return 12 * ns * ns - 2 * ir * (ir + 1) + ip;
}

void orc_hpx_ang2pix_many(int64_t ns, int64_t n, const double* lon_deg,
                          const double* lat_deg, int64_t* pix) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k) pix[k] = orc_hpx_ang2pix(ns, lon_deg[k], lat_deg[k]);
}

/* ------------------------------------------------------------------------ */
/* Gridding, Eq. (1).                                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t nx, ny;
  double lon0, lat0, dlon, dlat; /* degrees */
} orc_grid;

static void cell_centre(const orc_grid* g, int64_t ix, int64_t iy, double* lon, double* lat) {
  *lon = g->lon0 + ((double)ix - 0.5 * (double)(g->nx - 1)) * g->dlon;
  *lat = g->lat0 + ((double)iy - 0.5 * (double)(g->ny - 1)) * g->dlat;
}

/* great-circle distance in radians between two points given in degrees */
static double gc_dist(double lon1, double lat1, double lon2, double lat2) {
  double p1 = lat1 * ORC_DEG2RAD, p2 = lat2 * ORC_DEG2RAD;
  double dp = p2 - p1;
  double dl = (lon2 - lon1) * ORC_DEG2RAD;
  double s1 = sin(0.5 * dp), s2 = sin(0.5 * dl);
  double h = s1 * s1 + cos(p1) * cos(p2) * s2 * s2;
  if (h > 1.0) h = 1.0;
  return 2.0 * asin(sqrt(h));
}

double orc_sigma_rad(double fwhm_deg) {
  return fwhm_deg * ORC_DEG2RAD / (2.0 * sqrt(2.0 * log(2.0)));
}

/* Neumaier-compensated accumulation */
static inline void nsum_add(double* s, double* c, double x) {
  double t = *s + x;
  if (fabs(*s) >= fabs(x)) *c += (*s - t) + x; else *c += (x - t) + *s;
  *s = t;
}

/* One cell: accumulate the contributing pairs of a candidate list.  The
 * candidate list must contain every sample with d <= R (it may contain more).
 * Results: W (sum of weights), V[c] (normalised value, NaN when W == 0). */
static void grid_one_cell(double clon, double clat, int64_t ncand, const int64_t* cand,
                          const double* lon, const double* lat, const float* spec, int64_t C,
                          double R, double two_sig2, double* Vout, double* Wout,
                          int64_t* npair_out, double* num, double* numc) {
  double ws = 0.0, wc = 0.0;
  int64_t np = 0;
  for (int64_t c = 0; c < C; ++c) { num[c] = 0.0; numc[c] = 0.0; }
  for (int64_t q = 0; q < ncand; ++q) {
    int64_t k = cand ? cand[q] : q;
    double d = gc_dist(clon, clat, lon[k], lat[k]);
    if (!(d <= R)) continue;
    double w = exp(-(d * d) / two_sig2);
    ++np;
    nsum_add(&ws, &wc, w);
    const float* row = spec + k * C;
    for (int64_t c = 0; c < C; ++c) nsum_add(&num[c], &numc[c], w * (double)row[c]);
  }
  double W = ws + wc;
  *Wout = W;
  *npair_out = np;
  for (int64_t c = 0; c < C; ++c) Vout[c] = (W > 0.0) ? (num[c] + numc[c]) / W : NAN;
}

/*
 * All-pairs gridder: every (cell, sample) pair is tested.  The plain
 * definition of Eq. (1).  V is [C][ny][nx], W is [ny][nx], npairs (optional)
 * returns the number of contributing pairs.  Returns 0 on success.
 */
int orc_grid_allpairs(int64_t n, const double* lon, const double* lat, const float* spec,
                      int64_t C, const orc_grid* g, double fwhm_deg, double support_deg,
                      double* V, double* W, int64_t* npairs) {
  if (n < 0 || C < 1 || g->nx < 1 || g->ny < 1 || !(fwhm_deg > 0.0) || !(support_deg >= 0.0))
    return 1;
  double sig = orc_sigma_rad(fwhm_deg);
  double two_sig2 = 2.0 * sig * sig;
  double R = support_deg * ORC_DEG2RAD;
  int64_t G = (int64_t)g->nx * g->ny;
  int64_t total = 0;
#pragma omp parallel reduction(+ : total)
  {
    double* num = (double*)malloc(sizeof(double) * C);
    double* numc = (double*)malloc(sizeof(double) * C);
    double* vtmp = (double*)malloc(sizeof(double) * C);
#pragma omp for schedule(dynamic, 4)
    for (int64_t cell = 0; cell < G; ++cell) {
      double clon, clat, w;
      int64_t np;
      cell_centre(g, cell % g->nx, cell / g->nx, &clon, &clat);
      grid_one_cell(clon, clat, n, NULL, lon, lat, spec, C, R, two_sig2, vtmp, &w, &np, num, numc);
      W[cell] = w;
      for (int64_t c = 0; c < C; ++c) V[c * G + cell] = vtmp[c];
      total += np;
    }
    free(num); free(numc); free(vtmp);
  }
  if (npairs) *npairs = total;
  return 0;
}

/*
 * Bucketed search structure: samples are put in latitude bands of height
 * >= R and, inside a band, ordered by longitude (mod 360).  A cell needs the
 * bands overlapping [lat - R, lat + R] and, inside each, the longitudes within
 * the half-width asin(sin R / cos lat_max) (the whole band near the poles).
 * This only skips pairs with d > R; the exact test d <= R is still applied.
 */
typedef struct {
  int64_t n;
  double band_h;        /* band height, degrees */
  double lat_min;       /* latitude of the lower edge of band 0 */
  int64_t nbands;
  int64_t* band_start;  /* [nbands+1] offsets into idx */
  int64_t* idx;         /* sample indices, by (band, lon) */
  double* lon_sorted;   /* lon mod 360 of idx[] */
} orc_buckets;

typedef struct { double key; int64_t k; } orc_pair;

static int cmp_pair(const void* a, const void* b) {
  const orc_pair* x = (const orc_pair*)a;
  const orc_pair* y = (const orc_pair*)b;
  if (x->key < y->key) return -1;
  if (x->key > y->key) return 1;
  return (x->k < y->k) ? -1 : (x->k > y->k);
}

static double lon_mod(double lon) {
  double l = fmod(lon, 360.0);
  if (l < 0.0) l += 360.0;
  if (l >= 360.0) l -= 360.0;
  return l;
}

static int64_t band_of(const orc_buckets* b, double lat) {
  int64_t k = (int64_t)floor((lat - b->lat_min) / b->band_h);
  if (k < 0) k = 0;
  if (k >= b->nbands) k = b->nbands - 1;
  return k;
}

static int buckets_build(orc_buckets* b, int64_t n, const double* lon, const double* lat,
                         double support_deg) {
  memset(b, 0, sizeof(*b));
  b->n = n;
  double lo = 90.0, hi = -90.0;
  for (int64_t k = 0; k < n; ++k) {
    if (lat[k] < lo) lo = lat[k];
    if (lat[k] > hi) hi = lat[k];
  }
  if (n == 0) { lo = 0.0; hi = 0.0; }
  b->band_h = support_deg > 1e-6 ? support_deg : 1e-6;
  b->lat_min = lo;
  b->nbands = (int64_t)floor((hi - lo) / b->band_h) + 1;
  if (b->nbands > 100000000) return 1;
  b->band_start = (int64_t*)calloc((size_t)b->nbands + 1, sizeof(int64_t));
  b->idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  b->lon_sorted = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  orc_pair* tmp = (orc_pair*)malloc(sizeof(orc_pair) * (size_t)(n > 0 ? n : 1));
  if (!b->band_start || !b->idx || !b->lon_sorted || !tmp) { free(tmp); return 1; }
  for (int64_t k = 0; k < n; ++k) b->band_start[band_of(b, lat[k]) + 1] += 1;
  for (int64_t j = 0; j < b->nbands; ++j) b->band_start[j + 1] += b->band_start[j];
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)b->nbands);
  for (int64_t j = 0; j < b->nbands; ++j) fill[j] = b->band_start[j];
  for (int64_t k = 0; k < n; ++k) {
    int64_t j = band_of(b, lat[k]);
    tmp[fill[j]].key = lon_mod(lon[k]);
    tmp[fill[j]].k = k;
    fill[j] += 1;
  }
  free(fill);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t j = 0; j < b->nbands; ++j)
    qsort(tmp + b->band_start[j], (size_t)(b->band_start[j + 1] - b->band_start[j]),
          sizeof(orc_pair), cmp_pair);
  for (int64_t k = 0; k < n; ++k) { b->idx[k] = tmp[k].k; b->lon_sorted[k] = tmp[k].key; }
  free(tmp);
  return 0;
}

static void buckets_free(orc_buckets* b) {
  free(b->band_start); free(b->idx); free(b->lon_sorted);
  memset(b, 0, sizeof(*b));
}

/* first position in [lo, hi) with lon_sorted >= x */
static int64_t lower_lon(const orc_buckets* b, int64_t lo, int64_t hi, double x) {
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (b->lon_sorted[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

/* Collect into cand[] every sample that may lie within R of (clon, clat).
 * Returns the count; cand must hold n entries. */
static int64_t buckets_candidates(const orc_buckets* b, double clon, double clat,
                                  double support_deg, int64_t* cand) {
  int64_t nc = 0;
  if (b->n == 0) return 0;
  double lat_lo = clat - support_deg, lat_hi = clat + support_deg;
  int64_t j0 = band_of(b, lat_lo), j1 = band_of(b, lat_hi);
  double latmax = fmax(fabs(lat_lo), fabs(lat_hi));
  double half = 361.0; /* whole band */
  if (latmax < 89.0) {
    double s = sin(support_deg * ORC_DEG2RAD) / cos(latmax * ORC_DEG2RAD);
    if (s < 1.0) half = asin(s) / ORC_DEG2RAD * 1.000001 + 1e-9;
  }
  for (int64_t j = j0; j <= j1; ++j) {
    int64_t a = b->band_start[j], e = b->band_start[j + 1];
    if (half >= 180.0) {
      for (int64_t q = a; q < e; ++q) cand[nc++] = b->idx[q];
      continue;
    }
    double c = lon_mod(clon);
    double lo = c - half, hi = c + half;
    /* up to two lon intervals after wrapping into [0, 360) */
    double ivl[2][2];
    int nint = 0;
    if (lo < 0.0) {
      ivl[nint][0] = lo + 360.0; ivl[nint][1] = 360.0; nint++;
      ivl[nint][0] = 0.0; ivl[nint][1] = hi; nint++;
    } else if (hi >= 360.0) {
      ivl[nint][0] = lo; ivl[nint][1] = 360.0; nint++;
      ivl[nint][0] = 0.0; ivl[nint][1] = hi - 360.0; nint++;
    } else {
      ivl[nint][0] = lo; ivl[nint][1] = hi; nint++;
    }
    for (int q = 0; q < nint; ++q) {
      int64_t s = lower_lon(b, a, e, ivl[q][0]);
      int64_t t = lower_lon(b, a, e, nextafter(ivl[q][1], 1e300));
      for (int64_t m = s; m < t; ++m) cand[nc++] = b->idx[m];
    }
  }
  return nc;
}

/*
 * Bucketed gridder for a list of cells (flat index iy*nx + ix).  V is
 * [ncells][C] (cell-major), W is [ncells], npair[cell] (optional) the number
 * of contributing pairs per cell.  Same sums as orc_grid_allpairs, reached
 * through a pruned candidate search.  Returns 0 on success.
 */
int orc_grid_cells(int64_t n, const double* lon, const double* lat, const float* spec, int64_t C,
                   const orc_grid* g, double fwhm_deg, double support_deg, int64_t ncells,
                   const int64_t* cells, double* V, double* W, int64_t* npair) {
  if (n < 0 || C < 1 || g->nx < 1 || g->ny < 1 || !(fwhm_deg > 0.0) || !(support_deg >= 0.0))
    return 1;
  orc_buckets b;
  if (buckets_build(&b, n, lon, lat, support_deg)) { buckets_free(&b); return 2; }
  double sig = orc_sigma_rad(fwhm_deg);
  double two_sig2 = 2.0 * sig * sig;
  double R = support_deg * ORC_DEG2RAD;
  int err = 0;
#pragma omp parallel
  {
    double* num = (double*)malloc(sizeof(double) * C);
    double* numc = (double*)malloc(sizeof(double) * C);
    int64_t* cand = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!num || !numc || !cand) {
#pragma omp atomic write
      err = 3;
    }
#pragma omp for schedule(dynamic, 1)
    for (int64_t q = 0; q < ncells; ++q) {
      if (err) continue;
      int64_t cell = cells[q];
      double clon, clat, w;
      int64_t np;
      cell_centre(g, cell % g->nx, cell / g->nx, &clon, &clat);
      int64_t nc = buckets_candidates(&b, clon, clat, support_deg, cand);
      grid_one_cell(clon, clat, nc, cand, lon, lat, spec, C, R, two_sig2, V + q * C, &w, &np,
                    num, numc);
      W[q] = w;
      if (npair) npair[q] = np;
    }
    free(num); free(numc); free(cand);
  }
  buckets_free(&b);
  return err;
}

/*
 * For each listed cell, the set of samples with d <= R (all-pairs search),
 * in increasing sample order.  Two-call protocol: with out == NULL only
 * counts[ncells] are written; then out (sum of counts entries, concatenated
 * per cell in list order) is filled.  Returns 0 on success.
 */
int orc_neighbours(int64_t n, const double* lon, const double* lat, const orc_grid* g,
                   double support_deg, int64_t ncells, const int64_t* cells, int64_t* counts,
                   const int64_t* offsets, int64_t* out) {
  double R = support_deg * ORC_DEG2RAD;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t q = 0; q < ncells; ++q) {
    double clon, clat;
    int64_t cell = cells[q];
    cell_centre(g, cell % g->nx, cell / g->nx, &clon, &clat);
    int64_t m = 0;
    for (int64_t k = 0; k < n; ++k) {
      if (gc_dist(clon, clat, lon[k], lat[k]) <= R) {
        if (out) out[offsets[q] + m] = k;
        ++m;
      }
    }
    counts[q] = m;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Eq. (1) at arbitrary cell centres, with the kernel shapes of Section 3.6  */
/* (iii) and per-channel flags.                                              */
/* ------------------------------------------------------------------------ */

/*
 * Kernel w(g, n) of a cell g and a sample n at great-circle distance d
 * (d <= R; pairs beyond R have w = 0):
 *   type 0  Gaussian              exp(-d^2 / (2 sigma^2)), sigma from fwhm_deg;
 *   type 1  elliptical Gaussian   exp(-d^2/2 [cos^2(b - pa) / sa^2 + sin^2(b - pa) / sb^2])
 *           with b the position angle (bearing, from north through east) of
 *           the sample seen from the cell, sa / sb the sigmas of the major
 *           (fwhm_deg) and minor (fwhm_minor_deg) axes and pa the position
 *           angle of the major axis (pa_deg);
 *   type 2  Gaussian-tapered sinc sinc(d / b) exp(-(d / a)^2), sinc(x) =
 *           sin(pi x) / (pi x), b = sinc_deg, a = taper_deg: the sinc that
 *           Section 3.6 (iii) names as the optimal kernel of infinite length,
 *           cut to finite length by a Gaussian taper.
 */
typedef struct {
  int32_t type;
  double fwhm_deg, fwhm_minor_deg, pa_deg, sinc_deg, taper_deg;
} orc_kernel;

/* initial bearing of (lon2, lat2) seen from (lon1, lat1), radians, east of north */
static double gc_bearing(double lon1, double lat1, double lon2, double lat2) {
  double p1 = lat1 * ORC_DEG2RAD, p2 = lat2 * ORC_DEG2RAD;
  double dl = (lon2 - lon1) * ORC_DEG2RAD;
  return atan2(sin(dl) * cos(p2), cos(p1) * sin(p2) - sin(p1) * cos(p2) * cos(dl));
}

static double kernel_weight(const orc_kernel* k, double d, double clon, double clat, double slon,
                            double slat) {
  if (k->type == 0) {
    double s = orc_sigma_rad(k->fwhm_deg);
    return exp(-(d * d) / (2.0 * s * s));
  }
  if (k->type == 1) {
    if (d == 0.0) return 1.0;
    double sa = orc_sigma_rad(k->fwhm_deg), sb = orc_sigma_rad(k->fwhm_minor_deg);
    double t = gc_bearing(clon, clat, slon, slat) - k->pa_deg * ORC_DEG2RAD;
    double ct = cos(t), st = sin(t);
    return exp(-0.5 * d * d * (ct * ct / (sa * sa) + st * st / (sb * sb)));
  }
  double x = d / (k->sinc_deg * ORC_DEG2RAD);
  double sinc = (x == 0.0) ? 1.0 : sin(ORC_PI * x) / (ORC_PI * x);
  double u = d / (k->taper_deg * ORC_DEG2RAD);
  return sinc * exp(-u * u);
}

static int kernel_valid(const orc_kernel* k) {
  if (k->type == 0) return k->fwhm_deg > 0.0;
  if (k->type == 1) return k->fwhm_deg > 0.0 && k->fwhm_minor_deg > 0.0 && isfinite(k->pa_deg);
  if (k->type == 2) return k->sinc_deg > 0.0 && k->taper_deg > 0.0;
  return 0;
}

/* One cell at (clon, clat) over a candidate list that holds every sample with
 * d <= R.  masked = 0: W[0] = sum of the weights, V[c] = U[c] / W[0].
 * masked = 1: a non-finite value s_n[c] is a flag -- sample n is left out of
 * channel c, numerator and weights alike -- so W[c] = sum over the unflagged
 * samples of channel c and V[c] = U[c] / W[c].  V is NaN where its W is 0. */
static void grid_one_point(double clon, double clat, int64_t ncand, const int64_t* cand,
                           const double* lon, const double* lat, const float* spec, int64_t C,
                           double R, const orc_kernel* k, int masked, double* Vout, double* Wout,
                           int64_t* npair_out, double* num, double* numc, double* ws,
                           double* wc) {
  int64_t np = 0;
  int64_t nw = masked ? C : 1;
  for (int64_t c = 0; c < C; ++c) { num[c] = 0.0; numc[c] = 0.0; }
  for (int64_t c = 0; c < nw; ++c) { ws[c] = 0.0; wc[c] = 0.0; }
  for (int64_t q = 0; q < ncand; ++q) {
    int64_t m = cand ? cand[q] : q;
    double d = gc_dist(clon, clat, lon[m], lat[m]);
    if (!(d <= R)) continue;
    double w = kernel_weight(k, d, clon, clat, lon[m], lat[m]);
    ++np;
    const float* row = spec + m * C;
    if (!masked) {
      nsum_add(&ws[0], &wc[0], w);
      for (int64_t c = 0; c < C; ++c) nsum_add(&num[c], &numc[c], w * (double)row[c]);
    } else {
      for (int64_t c = 0; c < C; ++c) {
        if (!isfinite(row[c])) continue;
        nsum_add(&ws[c], &wc[c], w);
        nsum_add(&num[c], &numc[c], w * (double)row[c]);
      }
    }
  }
  *npair_out = np;
  for (int64_t c = 0; c < nw; ++c) Wout[c] = ws[c] + wc[c];
  for (int64_t c = 0; c < C; ++c) {
    double W = Wout[masked ? c : 0];
    Vout[c] = (W != 0.0) ? (num[c] + numc[c]) / W : NAN;
  }
}

/*
 * Eq. (1) at ncells arbitrary cell centres (cell_lon/cell_lat, degrees): a
 * target grid given by the world coordinates of its pixel centres, as a
 * projected (WCS) map gives them.  allpairs = 1 tests every (cell, sample)
 * pair; 0 takes the candidates of the latitude-band search, which only skips
 * pairs with d > R.  V is [ncells][C]; W is [ncells] (masked = 0) or
 * [ncells][C] (masked = 1); npair[ncells] (optional) counts the samples
 * within R.  A cell centre that is not finite has no samples (W = 0, V =
 * NaN).  Returns 0 on success.
 */
int orc_grid_points(int64_t n, const double* lon, const double* lat, const float* spec,
                    int64_t C, int64_t ncells, const double* cell_lon, const double* cell_lat,
                    const orc_kernel* k, double support_deg, int masked, int allpairs, double* V,
                    double* W, int64_t* npair) {
  if (n < 0 || C < 1 || ncells < 0 || !(support_deg >= 0.0) || !kernel_valid(k)) return 1;
  orc_buckets b;
  memset(&b, 0, sizeof(b));
  if (!allpairs && buckets_build(&b, n, lon, lat, support_deg)) { buckets_free(&b); return 2; }
  double R = support_deg * ORC_DEG2RAD;
  int64_t nw = masked ? C : 1;
  int err = 0;
#pragma omp parallel
  {
    double* num = (double*)malloc(sizeof(double) * C);
    double* numc = (double*)malloc(sizeof(double) * C);
    double* ws = (double*)malloc(sizeof(double) * nw);
    double* wc = (double*)malloc(sizeof(double) * nw);
    int64_t* cand = allpairs ? NULL : (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!num || !numc || !ws || !wc || (!allpairs && !cand)) {
#pragma omp atomic write
      err = 3;
    }
#pragma omp for schedule(dynamic, 1)
    for (int64_t q = 0; q < ncells; ++q) {
      if (err) continue;
      double clon = cell_lon[q], clat = cell_lat[q];
      int64_t np = 0, nc = 0;
      if (isfinite(clon) && isfinite(clat)) {
        nc = allpairs ? n : buckets_candidates(&b, clon, clat, support_deg, cand);
      } else {
        clon = clat = 0.0;
      }
      grid_one_point(clon, clat, nc, allpairs ? NULL : cand, lon, lat, spec, C, R, k, masked,
                     V + q * C, W + q * nw, &np, num, numc, ws, wc);
      if (npair) npair[q] = np;
    }
    free(num); free(numc); free(ws); free(wc); free(cand);
  }
  if (!allpairs) buckets_free(&b);
  return err;
}

void orc_set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
