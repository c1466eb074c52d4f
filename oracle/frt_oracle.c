/*
 * FP64 CPU oracle for one time step of adaptive ray tracing of ionizing
 * photon packets through a uniform Cartesian grid (Cain & D'Aloisio,
 * "FlexRT I", §3 "Adaptive Ray Tracing Implementation" and §4.1 "Standard
 * Mode"), with the backward-Euler hydrogen update and photon ledger that the
 * GPU path also implements.
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may build, load or call this file.  It shares no code,
 * header, table or helper with the HIP library; the two see the same seeded
 * inputs and nothing else.
 *
 * Everything is IEEE double in cgs units (cm, s, photons), compiled without
 * fast-math.  Nothing is blocked, fused or reordered beyond what the method
 * states; rays are marched depth-first one at a time, which is one valid
 * order of an order-independent sum.
 *
 * What pins each function (the tests under tests/test_oracle_*.py):
 *   healpix_nest_center   count 12*4^l (Eq. Nray), nesting of children
 *                         4p+i (Eq. lhpx), ring latitudes and equal area
 *                         (Gorski et al. 2005), base-pixel golden table.
 *   shoemake_rotation     orthonormality, det=+1, equality with the
 *                         quaternion sandwich product, Haar angle law.
 *   march_one_ray         per-cell path lengths and deposits against an
 *                         independent slab-intersection computation and
 *                         exact exp(-tau) transmission; optically thin limit
 *                         (Eq. gamma_initial_subgrid); split radius against
 *                         the footprint definition (Eq. r_split).
 *   chemistry_be          residual of the implicit equation, alpha=0 closed
 *                         form, Gamma=0 recombination, dt->inf equilibrium
 *                         (Eq. equilibrium_condition), convergence to an
 *                         ODE solver (Eq. ion_balance_eqn).
 *   chemistry_avg         x(t) and <x> against an ODE solver and its
 *                         quadrature at fixed n_e (Eqs. xi_of_t, avg_xi),
 *                         alpha=0 exponential decay, dt->inf equilibrium.
 *   orc_step (averaged)   with alpha = C = 0 the iterated step ionizes as many
 *                         atoms as its last march absorbed photons (the
 *                         photon conservation of §4.1), to the iteration's
 *                         convergence; ledger closure.
 *   orc_step (generalized) the moving screen's front radius against photon
 *                         counting, R = (3 Ndot t / (4 pi (1+chi) n_H))^(1/3)
 *                         (no recombination, transparent ionized gas), ionized
 *                         atoms against front photons, Gamma in ionized gas
 *                         against the absorbed photons (V/(sigma lambda) atoms
 *                         per cell), equality with Standard Mode when
 *                         kappa = n_HI sigma_0 and x_ion = 1 (§4.2), closure.
 *   orc_step              photon ledger closure, Stromgren I-front
 *                         (Eqs. r_of_t, rS, trec), checkpoint equality.
 *   merge_carried         (§3.3 ray merging) photons conserved per bin, the
 *                         exempt set is the N_ex N_RT brightest packets, at
 *                         most 12 4^l_merge merged packets per cell, and every
 *                         merged packet equals a brute-force regrouping of
 *                         the packets before the merge (photon sums,
 *                         photon-weighted positions, distances and levels,
 *                         the merging pixel's direction); merging with every
 *                         packet exempt changes nothing.
 *   temperature_update    (§4.1, Eq. temp_evolution_standard) the Hubble
 *                         term alone gives T0 e^(-2 H t); without heating
 *                         or cooling n_tot T is kept as the gas ionizes; the
 *                         thermal energy gained equals the photo-heating,
 *                         which equals heat_ev times the photons HI absorbed
 *                         (the photon ledger; per bin along one ray,
 *                         exactly); the paper's Test 2 (front beyond the
 *                         isothermal radius, ionized gas near 1e4 K).
 *   orc_rates             alpha_B(1e4 K) is the paper's 2.59e-13; alpha_A
 *                         lies within 3% of an independent fit (Verner &
 *                         Ferland 1996) from 1e2 to 1e6 K and of the
 *                         textbook 4.18e-13 at 1e4 K; the other fits are
 *                         those of the papers it cites (Hui & Gnedin 1997,
 *                         Cen 1992), restated, and beyond the Test 2 check
 *                         their values are parity unpinned.
 *   orc_set_density       (the compression term of Eq. temp_evolution_standard)
 *                         T Delta^(-2/3) against an ODE solver along a path
 *                         of densities; a change of the mean alone keeps T;
 *                         a later step sees the new density exactly as a
 *                         grid loaded with it.
 *   reion_heat_per_recombination  (§4.2, Eq. analytical_heating_HI) the
 *                         mean energy above 1 Ryd of the photons HI absorbs
 *                         from the cut power law, by quadrature.
 *   ionized_temperature_update, mixed_temperature  (Generalized Opacity
 *                         Mode, §4.2) gas the front ionizes enters at
 *                         T_reion and mixes by volume with the older
 *                         ionized gas, which cools as e^(-2 H t) where the
 *                         radiative terms vanish; neutral cells keep T; the
 *                         equilibrium temperature of highly ionized gas is
 *                         the same from above and below and for any n_H and
 *                         Gamma (heating and cooling both scale as n_e^2),
 *                         rises as the spectrum hardens and lies between
 *                         1e4 and 1e5 K; without photons (Gamma = 0) the
 *                         Hubble term alone gives T0 e^(-2 H t).
 *   Whole-field values beyond these properties: parity unpinned (the paper
 *   prints no per-cell numbers).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_BINS 8

/* ---------------------------------------------------------------- params */
typedef struct {
    int nx, ny, nz;          /* cells per axis */
    double dx;               /* cell edge, cm */
    int n_bins;              /* frequency bins, 1..8 */
    double sigma[ORC_MAX_BINS]; /* HI cross-section per bin, cm^2 */
    double alpha_B;          /* case-B recombination coefficient, cm^3/s */
    double coll_ion;         /* collisional ionization coefficient, cm^3/s */
    int base_level;          /* HEALPix level of cast rays (l_hpx) */
    int max_level;           /* rays at this level never split */
    double n_ray_min;        /* N_ray^min of Eq. r_split */
    double flux_floor;       /* drop when sum N < floor * sum N_init; 0 = off */
    double max_dist;         /* drop at this distance from the source, cm; 0 = off */
    double c_ray;            /* packet speed, cm/s; +inf = finish within the step */
    int n_chunks;            /* fixed source chunking for a deterministic sum */
    int chem_iterations;     /* 0: backward Euler; K >= 1: the time-averaged update
                                of §4.1 with K marches per step */
    int opacity_mode;        /* 0: Standard Mode (§4.1); 1: Generalized Opacity Mode
                                (§4.2): kappa is the ionized phase's absorption
                                coefficient at sigma_0, x = 1 - x_ion the neutral
                                volume fraction behind a moving screen */
    double he_chi;           /* chi of Eq. dxidt (helium singly ionized with H) */
    int merge;               /* 1: merge the carried packets at the end of each step (§3.3) */
    int merge_level;         /* l_merge: level of each cell's merging HEALPix sphere */
    double merge_exempt;     /* N_ex: floor(N_ex N_RT) brightest packets are exempt */
    int temperature;         /* 1: T evolves (§4.1, Eq. temp_evolution_standard) and the
                                recombination and collisional ionization rates follow it
                                (Generalized Opacity Mode: the ionized part's T, §4.2);
                                0: alpha_B and coll_ion as given */
    double heat_ev[ORC_MAX_BINS]; /* mean energy above 13.6 eV left in the gas per photon
                                of each bin that HI absorbs, eV */
    double hubble;           /* H(z) of the adiabatic cooling term, 1/s (0: none) */
    double cmb_z;            /* redshift of the CMB for Compton cooling (< 0: none) */
    double t_reion;          /* Generalized Opacity Mode: temperature of gas the front
                                ionizes, K */
    double spectral_index;   /* Generalized Opacity Mode: power-law index alpha of the
                                ionizing spectrum in its photo-heating estimate */
} orc_params;

typedef struct {
    double emitted, absorbed_HI, absorbed_sub, escaped, dropped, in_flight;
    long long crossings, rays_emitted, splits, n_escaped, n_dropped, n_in_flight;
    double absorbed_front;   /* photons stopped by I-fronts (Generalized Opacity Mode) */
    double merge_residual;   /* photons held before minus after the merges (rounding only) */
    long long merges, rays_merged; /* merged packets made, and packets merged into them */
    double front_excess;     /* photons stopped at a front beyond the neutral atoms its
                                cell had left (they ionize nothing); absorbed_front
                                counts only the photons that ionized atoms */
    double heat_in;          /* photo-heating energy given to the gas, erg (temperature on) */
} orc_ledger;

/* Photon totals are sums of up to ~1e9 terms; they are accumulated with
 * Neumaier's compensated summation so that the ledger closes to rounding
 * level whatever the number of rays. */
typedef struct { double s, c; } csum;

static void csum_add(csum* a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}

static double csum_get(const csum* a) { return a->s + a->c; }

typedef struct {
    csum emitted, absorbed_HI, absorbed_sub, escaped, dropped, front;
    long long crossings, rays_emitted, splits, n_escaped, n_dropped, n_in_flight;
} chunk_ledger;

/* One ray (photon packet).  Its position is always origin + r * dir:
 * children are re-centred on their own pixel directions at the split radius
 * (§3.2), so the distance from the origin fully fixes the position. */
typedef struct {
    int src;                 /* emitting source, or -1 for a merged packet */
    int level;
    long long pix;
    double dir[3];
    double R[9];             /* rotation of the emitting step, inherited (§3.1, §3.2) */
    double origin[3];        /* the point the packet travels from, cm: its source, or the
                                virtual origin of a merged packet (position - r dir) */
    double r;                /* distance travelled from the source, cm */
    double r_stop;           /* distance at which this step's travel budget ends */
    double N[ORC_MAX_BINS];      /* photons carried per bin */
    double Ninit[ORC_MAX_BINS];  /* photons at casting, divided by 4 per split */
} orc_ray;

typedef struct {
    orc_ray* v;
    long long n, cap;
} orc_vec;

typedef struct {
    orc_params p;
    long long ncell;
    double* nH;              /* cm^-3 */
    double* kappa;           /* sub-grid absorption coefficient, 1/cm */
    double* x;               /* neutral fraction x_HI */
    double* gamma;           /* last step's photo-ionization rate, 1/s */
    double* T;               /* gas temperature, K (1e4 until set) */
    int nsrc;
    double* src_pos;         /* nsrc*3, cm */
    double* ndot;            /* nsrc*n_bins, photons/s */
    orc_vec carried;         /* packets carried into the next step, in a fixed order */
    orc_ledger L;
    long long step;
    long long last_crossings;
} orc_state;

/* ------------------------------------------------------------- vectors */
static int vec_push(orc_vec* a, const orc_ray* r)
{
    if (a->n == a->cap) {
        long long nc = a->cap ? 2 * a->cap : 64;
        orc_ray* nv = (orc_ray*)realloc(a->v, (size_t)nc * sizeof(orc_ray));
        if (!nv) return -1;
        a->v = nv;
        a->cap = nc;
    }
    a->v[a->n++] = *r;
    return 0;
}

/* ------------------------------------------------------------- HEALPix */
/* Face layout of the 12 base pixels (Gorski et al. 2005, Fig. 3): the ring
 * coordinate of each face's southern vertex in units of Nside, and the
 * longitude of its centre in units of pi/4. */
static const int FACE_RING[12] = {2, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4};
static const int FACE_LON[12] = {1, 3, 5, 7, 0, 2, 4, 6, 1, 3, 5, 7};

/* Take every second bit of v starting at bit `first` (0 or 1). */
static long long take_alternate_bits(long long v, int first)
{
    long long out = 0;
    int k = 0;
    for (int b = first; b < 62; b += 2, k++)
        if ((v >> b) & 1LL) out |= (1LL << k);
    return out;
}

/* Map continuous face coordinates (a, b) in [0,1]^2 of face f onto the unit
 * sphere.  rho = FACE_RING[f] - a - b is the ring coordinate (0 at the north
 * pole, 4 at the south pole, in units of Nside); the polar caps (rho<1,
 * rho>3) and the equatorial belt use the two HEALPix projections. */
static void face_to_sphere(int f, double a, double b, double out[3])
{
    double rho = FACE_RING[f] - a - b;
    double z, width;
    if (rho < 1.0) {
        z = 1.0 - rho * rho / 3.0;
        width = rho;
    } else if (rho > 3.0) {
        double s = 4.0 - rho;
        z = s * s / 3.0 - 1.0;
        width = s;
    } else {
        z = (2.0 - rho) * 2.0 / 3.0;
        width = 1.0;
    }
    double phi = (M_PI / 4.0) * (FACE_LON[f] + (a - b) / width);
    double st = sqrt((1.0 - z) * (1.0 + z));
    out[0] = st * cos(phi);
    out[1] = st * sin(phi);
    out[2] = z;
}

/* Unit vector of the centre of NESTED pixel p at level l (Nside = 2^l). */
void healpix_nest_center(int level, long long p, double out[3])
{
    long long nside = 1LL << level;
    long long per_face = nside * nside;
    int f = (int)(p / per_face);
    long long q = p % per_face;
    long long ia = take_alternate_bits(q, 0);
    long long ib = take_alternate_bits(q, 1);
    face_to_sphere(f, (ia + 0.5) / (double)nside, (ib + 0.5) / (double)nside, out);
}

/* Inverse map for tests: the NESTED pixel containing unit vector v.  Each of
 * the 12 faces is tried; the one whose face coordinates fall in [0,1)^2
 * holds the point. */
long long healpix_nest_pixel(int level, const double v[3])
{
    long long nside = 1LL << level;
    double z = v[2];
    double phi = atan2(v[1], v[0]);
    if (phi < 0) phi += 2.0 * M_PI;
    double rho, width;
    if (z > 2.0 / 3.0) {
        rho = sqrt(3.0 * (1.0 - z));
        width = rho;
    } else if (z < -2.0 / 3.0) {
        width = sqrt(3.0 * (1.0 + z));
        rho = 4.0 - width;
    } else {
        rho = 2.0 - 1.5 * z;
        width = 1.0;
    }
    for (int f = 0; f < 12; f++) {
        double lon = phi / (M_PI / 4.0) - FACE_LON[f];
        while (lon >= 4.0) lon -= 8.0;
        while (lon < -4.0) lon += 8.0;
        double s = FACE_RING[f] - rho;     /* a + b */
        double d = lon * width;            /* a - b */
        double a = 0.5 * (s + d), b = 0.5 * (s - d);
        if (a >= 0.0 && a < 1.0 && b >= 0.0 && b < 1.0) {
            long long ia = (long long)floor(a * nside), ib = (long long)floor(b * nside);
            long long q = 0;
            for (int k = 0; k < 31; k++) {
                q |= ((ia >> k) & 1LL) << (2 * k);
                q |= ((ib >> k) & 1LL) << (2 * k + 1);
            }
            return (long long)f * nside * nside + q;
        }
    }
    return -1;
}

/* ------------------------------------------------------------ rotation */
/* Uniform random rotation from three uniforms (Shoemake 1992, "Uniform
 * random rotations", Graphics Gems III): unit quaternion
 *   x = sqrt(1-u1) sin(2 pi u2), y = sqrt(1-u1) cos(2 pi u2),
 *   z = sqrt(u1) sin(2 pi u3),   w = sqrt(u1) cos(2 pi u3),
 * turned into the row-major matrix of v -> q v q*.  §3.1 rotates each
 * source's sphere by random angles every step; children keep them (§3.2). */
void shoemake_rotation(const double u[3], double R[9])
{
    double s1 = sqrt(1.0 - u[0]), s2 = sqrt(u[0]);
    double x = s1 * sin(2.0 * M_PI * u[1]);
    double y = s1 * cos(2.0 * M_PI * u[1]);
    double z = s2 * sin(2.0 * M_PI * u[2]);
    double w = s2 * cos(2.0 * M_PI * u[2]);
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

static void set_direction(orc_ray* ray)
{
    double n[3];
    healpix_nest_center(ray->level, ray->pix, n);
    for (int i = 0; i < 3; i++)
        ray->dir[i] = ray->R[3 * i] * n[0] + ray->R[3 * i + 1] * n[1] + ray->R[3 * i + 2] * n[2];
}

/* ------------------------------------------------------------ geometry */
/* Eq. r_split: distance from the source at which a level-l ray splits. */
double split_radius(double dx, int level, double n_ray_min)
{
    return dx * ldexp(1.0, level) * sqrt(3.0 / (M_PI * n_ray_min));
}

/* Cell holding point `pos` for a ray moving along `dir`: floor per axis, and
 * a point exactly on a cell face belongs to the cell the ray is entering. */
static void locate(const orc_params* P, const double pos[3], const double dir[3], long long c[3])
{
    for (int a = 0; a < 3; a++) {
        double u = pos[a] / P->dx;
        double f = floor(u);
        if (u == f && dir[a] < 0.0) f -= 1.0;
        c[a] = (long long)f;
    }
}

static int inside(const orc_params* P, const long long c[3])
{
    return c[0] >= 0 && c[0] < P->nx && c[1] >= 0 && c[1] < P->ny && c[2] >= 0 && c[2] < P->nz;
}

static double sum_bins(const double* v, int n)
{
    double s = 0.0;
    for (int i = 0; i < n; i++) s += v[i];
    return s;
}

/* ---------------------------------------------------------------- march */
typedef struct {
    const orc_state* S;
    const double* nHI;       /* start-of-step neutral density snapshot */
    double* gamma;           /* this chunk's photo-ionization accumulator */
    chunk_ledger* L;
    orc_vec* stack;          /* depth-first work list */
    orc_vec* flight_out;     /* packets that end the step in flight */
    double inv_vdt;          /* 1 / (V_cell dt) */
    const double* xion;      /* Generalized Opacity Mode: start-of-step ionized fraction */
    const double* kappa;     /* Generalized Opacity Mode: the ionized gas's absorption coefficient at sigma_0 */
    double* front;           /* this chunk's photons stopped at each cell's I-front */
    double* heat;            /* this chunk's photo-heating per cell, eV (temperature on), or NULL */
} march_ctx;

/* March one ray from its current radius until it is absorbed below the floor,
 * reaches the distance cap, splits, leaves the box, or spends its travel
 * budget (§3.1 packets, §3.2 splitting, §4.1 deposition).  Per segment of
 * length ds in cell i and bin nu:
 *   tau     = (n_HI sigma_nu + kappa) ds                    (Eq. tau_cell)
 *   N_out   = N_in exp(-tau)
 *   Gamma_i += N_in sigma_nu ds phi(tau) / (V dt),  phi(t) = (1 - e^-t)/t
 * which equals N_in (1 - e^-tau)/(n_HI V dt) x (HI share of tau), i.e.
 * Eq. gamma_initial_standard when kappa = 0 and Eq. gamma_avg_subgrid with
 * lambda = 1/(n_HI sigma + kappa), and tends to Eq. gamma_initial_subgrid
 * as tau -> 0.  With the temperature on, each bin's photons absorbed by HI
 * (the HI share of N_in - N_out) leave heat_ev of that bin each in the cell
 * (photo-heating of Eq. temp_evolution_standard).
 *
 * Generalized Opacity Mode (§4.2): a cell is an ionized part of volume
 * fraction x_ion with absorption coefficient kappa_nu = kappa sigma_nu /
 * sigma_0 and a neutral part behind an infinitely thin front (the moving
 * screen).  A segment crosses the ionized part first, over x_ion ds:
 *   tau     = kappa_nu x_ion ds
 *   Gamma_i += N_in sigma_nu ds phi(tau) / (V dt)
 * which is Eq. gamma_avg_subgrid with ds -> x_ion ds and V -> x_ion V; in a
 * cell that is not fully ionized the photons left then reach the front and
 * are absorbed there (they drive Eq. dxidt), ending the packet. */
static void march_one_ray(march_ctx* M, orc_ray* ray)
{
    const orc_params* P = &M->S->p;
    const int nb = P->n_bins;
    const double* o = ray->origin;
    const double r_split = (ray->level < P->max_level) ? split_radius(P->dx, ray->level, P->n_ray_min) : INFINITY;
    const double r_cap = (P->max_dist > 0.0) ? P->max_dist : INFINITY;
    double pos[3];
    long long c[3];
    for (int a = 0; a < 3; a++) pos[a] = o[a] + ray->r * ray->dir[a];
    locate(P, pos, ray->dir, c);
    if (!inside(P, c)) {
        csum_add(&M->L->escaped, sum_bins(ray->N, nb));
        M->L->n_escaped++;
        return;
    }
    for (;;) {
        /* distance from the source to the face through which the ray leaves
         * the current cell; lowest axis first on ties */
        double r_face = INFINITY;
        int axis = -1;
        for (int a = 0; a < 3; a++) {
            double rf = INFINITY;
            if (ray->dir[a] > 0.0) rf = ((double)(c[a] + 1) * P->dx - o[a]) / ray->dir[a];
            else if (ray->dir[a] < 0.0) rf = ((double)c[a] * P->dx - o[a]) / ray->dir[a];
            if (rf < r_face) { r_face = rf; axis = a; }
        }
        double r_end = r_face;
        if (r_split < r_end) r_end = r_split;
        if (r_cap < r_end) r_end = r_cap;
        if (ray->r_stop < r_end) r_end = ray->r_stop;
        if (r_end < ray->r) r_end = ray->r;
        double ds = r_end - ray->r;
        if (ds > 0.0 && P->opacity_mode == 1) {
            long long i = c[0] + (long long)P->nx * (c[1] + (long long)P->ny * c[2]);
            const double xi = M->xion[i], kap = M->kappa[i];
            double g = 0.0;
            for (int k = 0; k < nb; k++) {
                double tau = kap * (P->sigma[k] / P->sigma[0]) * xi * ds;
                double Nin = ray->N[k];
                double Nout = Nin * exp(-tau);
                double phi = (tau > 0.0) ? -expm1(-tau) / tau : 1.0;
                g += Nin * P->sigma[k] * ds * phi;
                csum_add(&M->L->absorbed_HI, Nin - Nout);
                ray->N[k] = Nout;
            }
            M->gamma[i] += g * M->inv_vdt;
            M->L->crossings++;
            if (xi < 1.0) {
                const double left = sum_bins(ray->N, nb);
                M->front[i] += left;
                csum_add(&M->L->front, left);
                return;
            }
        } else if (ds > 0.0) {
            long long i = c[0] + (long long)P->nx * (c[1] + (long long)P->ny * c[2]);
            double nhi = M->nHI[i], kap = M->S->kappa[i];
            double g = 0.0, heat = 0.0;
            for (int k = 0; k < nb; k++) {
                double tau_h = nhi * P->sigma[k] * ds;
                double tau = tau_h + kap * ds;
                double Nin = ray->N[k];
                double Nout = Nin * exp(-tau);
                double phi = (tau > 0.0) ? -expm1(-tau) / tau : 1.0;
                g += Nin * P->sigma[k] * ds * phi;
                double dA = Nin - Nout;
                if (tau > 0.0) {
                    csum_add(&M->L->absorbed_HI, dA * (tau_h / tau));
                    csum_add(&M->L->absorbed_sub, dA * ((kap * ds) / tau));
                    heat += P->heat_ev[k] * dA * (tau_h / tau);
                }
                ray->N[k] = Nout;
            }
            M->gamma[i] += g * M->inv_vdt;
            if (M->heat) M->heat[i] += heat;
            M->L->crossings++;
        }
        ray->r = r_end;
        /* end states, in this order */
        if (ray->r >= r_cap) {
            csum_add(&M->L->dropped, sum_bins(ray->N, nb));
            M->L->n_dropped++;
            return;
        }
        if (P->flux_floor > 0.0 && sum_bins(ray->N, nb) < P->flux_floor * sum_bins(ray->Ninit, nb)) {
            csum_add(&M->L->dropped, sum_bins(ray->N, nb));
            M->L->n_dropped++;
            return;
        }
        if (ray->r >= r_split) {
            /* four children (Eq. lhpx), photons shared equally, re-centred on
             * their own pixel directions at this radius, same rotation */
            M->L->splits++;
            for (int k = 3; k >= 0; k--) {
                orc_ray ch = *ray;
                ch.level = ray->level + 1;
                ch.pix = 4 * ray->pix + k;
                for (int b = 0; b < nb; b++) {
                    ch.N[b] = ray->N[b] / 4.0;
                    ch.Ninit[b] = ray->Ninit[b] / 4.0;
                }
                set_direction(&ch);
                vec_push(M->stack, &ch);
            }
            return;
        }
        if (ray->r >= r_face) {
            c[axis] += (ray->dir[axis] > 0.0) ? 1 : -1;
            if (!inside(P, c)) {
                csum_add(&M->L->escaped, sum_bins(ray->N, nb));
                M->L->n_escaped++;
                return;
            }
        }
        if (ray->r >= ray->r_stop) {
            M->L->n_in_flight++;
            vec_push(M->flight_out, ray);
            return;
        }
    }
}

static void drain(march_ctx* M)
{
    while (M->stack->n > 0) {
        orc_ray ray = M->stack->v[--M->stack->n];
        march_one_ray(M, &ray);
    }
}

/* ----------------------------------------------------------- chemistry */
/* Backward-Euler update of the neutral fraction x = n_HI/n_H for pure H with
 * n_e = n_HII = n_H (1-x), discretizing Eq. ion_balance_eqn (collisional
 * term read as C n_e n_HI):
 *   x' - x = dt [ -Gamma x' - C n_H (1-x') x' + alpha n_H (1-x')^2 ]
 * i.e. a x'^2 + b x' + c = 0 with a = dt n_H (alpha + C),
 * b = -(1 + dt (Gamma + 2 alpha n_H + C n_H)), c = x + alpha n_H dt.
 * The root in [0,1] is the smaller one, written as 2c / (-b + sqrt(b^2-4ac))
 * so that it stays accurate when x << 1 and when a = 0. */
double chemistry_be(double x, double gamma, double nH, double alpha, double coll, double dt)
{
    double a = dt * nH * (alpha + coll);
    double b = -(1.0 + dt * (gamma + 2.0 * alpha * nH + coll * nH));
    double c = x + alpha * nH * dt;
    double disc = b * b - 4.0 * a * c;
    if (disc < 0.0) disc = 0.0;
    return 2.0 * c / (-b + sqrt(disc));
}

/* Time-averaged update of §4.1 (Eqs. xi_of_t, xeq, ti, avg_xi), for the
 * neutral fraction x = 1 - x_i, which follows the same linear equation once
 * the electron density n_e is held fixed over the step:
 *   dx/dt = alpha n_e (1 - x) - (Gamma + C n_e) x        (Eq. ion_balance_eqn / n_H)
 * with the equilibrium x_eq = alpha n_e / R and time constant t_i = 1 / R,
 * R = Gamma + C n_e + alpha n_e.  Then
 *   x(dt) = x_eq + (x0 - x_eq) exp(-dt/t_i)
 *   <x>   = x_eq + (x0 - x_eq) (1 - exp(-dt/t_i)) t_i / dt.
 * Returns <x> and stores x(dt) in *x_end.  With R = 0 nothing changes. */
double chemistry_avg(double x0, double gamma, double ne, double alpha, double coll, double dt, double* x_end)
{
    const double R = gamma + coll * ne + alpha * ne;
    const double y = R * dt;
    if (!(y > 0.0)) {
        *x_end = x0;
        return x0;
    }
    const double xeq = alpha * ne / R;
    *x_end = xeq + (x0 - xeq) * exp(-y);
    return xeq + (x0 - xeq) * (-expm1(-y) / y);
}

/* ---------------------------------------------------------- temperature */
/* Rates of pure hydrogen gas at temperature T (K) that the temperature
 * evolution uses (§4.1 cites Hui & Gnedin 1997 for them), with
 * lambda = 2 T_HI / T and T_HI = 157807 K:
 *   [0] alpha_B, case-B recombination coefficient, cm^3/s
 *       (Hui & Gnedin 1997 fit: 2.753e-14 lambda^1.5 / (1 + (lambda/2.740)^0.407)^2.242)
 *   [1] C_HI, collisional ionization coefficient, cm^3/s
 *       (21.11 T^-1.5 e^(-lambda/2) lambda^-1.089 / (1 + (lambda/0.354)^0.874)^1.101)
 *   [2] case-B recombination cooling coefficient, erg cm^3/s (times n_e n_HII)
 *       (3.435e-30 T lambda^1.970 / (1 + (lambda/2.250)^0.376)^3.720)
 *   [3] collisional ionization cooling, erg cm^3/s (times n_e n_HI): the
 *       ionization energy k T_HI per collisional ionization, k T_HI C_HI
 *   [4] collisional excitation cooling, erg cm^3/s (times n_e n_HI)
 *       (Cen 1992: 7.5e-19 e^(-118348/T) / (1 + (T/1e5)^0.5))
 *   [5] free-free cooling, erg cm^3/s (times n_e n_HII)
 *       (1.42e-27 g_ff T^0.5, g_ff = 1.1 + 0.34 exp(-(5.5 - log10 T)^2 / 3))
 *   [6] alpha_A, case-A recombination coefficient, cm^3/s
 *       (Hui & Gnedin 1997 fit: 1.269e-13 lambda^1.503 / (1 + (lambda/0.522)^0.470)^1.923)
 * Compton cooling off the CMB is 4 sigma_T a k T_CMB^4 (T - T_CMB) n_e /
 * (m_e c) with T_CMB = 2.725 (1 + z) K. */
#define ORC_T_HI 157807.0
#define ORC_K_B 1.380649e-16
#define ORC_EV 1.602176634e-12
void orc_rates(double T, double* out)
{
    const double lam = 2.0 * ORC_T_HI / T;
    out[0] = 2.753e-14 * pow(lam, 1.5) / pow(1.0 + pow(lam / 2.740, 0.407), 2.242);
    out[1] = 21.11 * pow(T, -1.5) * exp(-0.5 * lam) * pow(lam, -1.089) / pow(1.0 + pow(lam / 0.354, 0.874), 1.101);
    out[2] = 3.435e-30 * T * pow(lam, 1.970) / pow(1.0 + pow(lam / 2.250, 0.376), 3.720);
    out[3] = ORC_K_B * ORC_T_HI * out[1];
    out[4] = 7.5e-19 * exp(-118348.0 / T) / (1.0 + sqrt(T / 1e5));
    const double lg = 5.5 - log10(T);
    out[5] = 1.42e-27 * (1.1 + 0.34 * exp(-lg * lg / 3.0)) * sqrt(T);
    out[6] = 1.269e-13 * pow(lam, 1.503) / pow(1.0 + pow(lam / 0.522, 0.470), 1.923);
}

static double compton_coefficient(void)
{
    const double sigma_T = 6.6524587321e-25, a_rad = 7.565733e-15, m_e = 9.1093837015e-28, c = 2.99792458e10;
    const double T0 = 2.725;
    return 4.0 * sigma_T * a_rad * ORC_K_B * T0 * T0 * T0 * T0 / (m_e * c);
}

/* Net heating minus cooling, erg/cm^3/s, of a cell with n_H, neutral
 * fraction x and photo-heating h (erg/cm^3/s) at temperature T. */
static double net_heating(const orc_params* P, double T, double nH, double x, double h)
{
    double r[7];
    orc_rates(T, r);
    const double nHI = nH * x, ne = nH * (1.0 - x), nHII = ne;
    double L = r[2] * ne * nHII + (r[3] + r[4]) * ne * nHI + r[5] * ne * nHII;
    if (P->cmb_z >= 0.0) {
        const double z1 = 1.0 + P->cmb_z;
        L += compton_coefficient() * z1 * z1 * z1 * z1 * (T - 2.725 * z1) * ne;
    }
    return h - L;
}

/* Temperature over one step (§4.1, Eq. temp_evolution_standard, static
 * density: no compression term) once the neutral fraction went from x0 to
 * x1, for pure H (n_tot = n_H (2 - x)), in three parts taken in turn:
 *  - the particle-number term -T/n_tot dn_tot/dt, exactly: n_tot T is kept,
 *    T -> T n_tot(x0) / n_tot(x1);
 *  - the Hubble term -2 H T, exactly: T -> T e^(-2 H dt);
 *  - heating minus cooling, dT/dt = 2 (H - Lambda(T)) / (3 k n_tot), with
 *    the step's photo-heating H and x = x1, in sub-steps that change T by at
 *    most a tenth, each the exact solution of the equation linearized about
 *    its start (T += f (e^(f' h) - 1) / f', f' from a relative difference of
 *    1e-6 in T), at most 4096 sub-steps, T >= 1 K.
 * h_heat is the step's photo-heating, erg/cm^3/s. */
double temperature_update(const orc_params* P, double T, double nH, double x0, double x1, double h_heat, double dt)
{
    const double nt0 = nH * (2.0 - x0), nt1 = nH * (2.0 - x1);
    if (nt1 > 0.0) T *= nt0 / nt1;
    if (P->hubble > 0.0) T *= exp(-2.0 * P->hubble * dt);
    if (!(nt1 > 0.0)) return T;
    const double cth = 2.0 / (3.0 * ORC_K_B * nt1);
    double t = 0.0;
    for (int k = 0; k < 4096 && t < dt; k++) {
        const double f = cth * net_heating(P, T, nH, x1, h_heat);
        const double Te = T * (1.0 + 1e-6);
        const double fp = (cth * net_heating(P, Te, nH, x1, h_heat) - f) / (Te - T);
        double h = dt - t;
        if (fabs(f) * h > 0.1 * T) h = 0.1 * T / fabs(f);
        const double y = fp * h;
        T += (fabs(y) > 1e-8) ? f * expm1(y) / fp : f * h;
        if (T < 1.0) T = 1.0;
        t += h;
    }
    return T;
}

/* Generalized Opacity Mode (§4.2, after Eq. dxidt): T is the temperature of
 * each cell's ionized part.  Its n_HI is not known, so the rates that need
 * it take photo-ionization equilibrium with the step's Gamma of the ionized
 * gas (Eqs. equilibrium_condition and subgrid_nHI with alpha_B(T)):
 * y = n_HI / n_H = min(1, alpha_B(T) n_H / Gamma), y = 1 where Gamma = 0,
 * n_e = n_HII = n_H (1 - y), n_tot = n_H (2 - y).  The photo-heating is that
 * of Eq. analytical_heating_HI, pure H:
 *   H = E_HI q alpha_A(T) n_e n_HII,  q = s/(s-1) (1 - 4^(1-s)) / (1 - 4^-s) - 1,
 * s = alpha + beta, beta = 2.75 (sigma_HI ~ nu^-beta), alpha the spectral
 * index, E_HI = 1 Ryd: q E_HI is the mean energy above E_HI of the photons
 * that HI absorbs from a power law nu^-alpha cut off at 4 Ryd.  The cooling
 * is Standard Mode's. */
#define ORC_RYD_EV 13.605693122994
double reion_heat_per_recombination(double spectral_index)
{
    const double s = spectral_index + 2.75;
    const double q = s / (s - 1.0) * (1.0 - pow(4.0, 1.0 - s)) / (1.0 - pow(4.0, -s)) - 1.0;
    return q * ORC_RYD_EV * ORC_EV;
}

/* (H - Lambda) 2 / (3 k n_tot), K/s, of the ionized part of a cell at T. */
static double ionized_dTdt(const orc_params* P, double T, double nH, double gamma)
{
    double r[7];
    orc_rates(T, r);
    const double y = (gamma > r[0] * nH) ? r[0] * nH / gamma : 1.0;
    const double ne = nH * (1.0 - y), nHI = nH * y;
    const double H = reion_heat_per_recombination(P->spectral_index) * r[6] * ne * ne;
    double L = (r[2] + r[5]) * ne * ne + (r[3] + r[4]) * ne * nHI;
    if (P->cmb_z >= 0.0) {
        const double z1 = 1.0 + P->cmb_z;
        L += compton_coefficient() * z1 * z1 * z1 * z1 * (T - 2.725 * z1) * ne;
    }
    return 2.0 * (H - L) / (3.0 * ORC_K_B * nH * (2.0 - y));
}

/* Temperature of the ionized part of a cell over one step: the Hubble term
 * exactly (T -> T e^(-2 H dt)), then dT/dt = ionized_dTdt in the sub-steps
 * of temperature_update (a tenth change in T at most, each the exact
 * solution of the equation linearized about its start, at most 4096,
 * T >= 1 K).  Static density: no compression term; y is an equilibrium
 * value, so there is no particle-number term. */
double ionized_temperature_update(const orc_params* P, double T, double nH, double gamma, double dt)
{
    if (P->hubble > 0.0) T *= exp(-2.0 * P->hubble * dt);
    if (!(nH > 0.0)) return T;
    double t = 0.0;
    for (int k = 0; k < 4096 && t < dt; k++) {
        const double f = ionized_dTdt(P, T, nH, gamma);
        const double Te = T * (1.0 + 1e-6);
        const double fp = (ionized_dTdt(P, Te, nH, gamma) - f) / (Te - T);
        double h = dt - t;
        if (fabs(f) * h > 0.1 * T) h = 0.1 * T / fabs(f);
        const double yl = fp * h;
        T += (fabs(yl) > 1e-8) ? f * expm1(yl) / fp : f * h;
        if (T < 1.0) T = 1.0;
        t += h;
    }
    return T;
}

/* A cell's temperature at the end of a step in which its ionized fraction
 * went from xi0 to xi1: the part ionized before the step evolved at T_ion,
 * the part ionized during it at T_reion, mixed by volume (both are ionized
 * gas of the cell's n_H, so by particle number too); a cell with no ionized
 * gas keeps its temperature. */
static double mixed_temperature(const orc_params* P, double T, double nH, double gamma, double xi0, double xi1,
                                double dt)
{
    const double T_ion = xi0 > 0.0 ? ionized_temperature_update(P, T, nH, gamma, dt) : T;
    if (xi1 > xi0) return (xi0 * T_ion + (xi1 - xi0) * P->t_reion) / xi1;
    return xi0 > 0.0 ? T_ion : T;
}

/* ------------------------------------------------------------- merging */
/* §3.3: at the end of a step the carried packets are ranked by their
 * photons; the floor(N_ex N_RT) brightest are exempt (every packet with at
 * least the photons of the last of them: ties at the threshold are all
 * exempt).  The others are grouped by the cell they are in and by the pixel,
 * on a HEALPix sphere of level l_merge rotated at random for that cell and
 * step, that holds their direction.  A group of one is left as it is; a
 * larger group becomes one packet with the summed photons of every bin,
 * travelling along the pixel's centre, its position, distance from its origin
 * and level the photon-weighted means of its members' (the level rounded to
 * the nearest integer), its initial photons its photons at the merge.  So
 * that it moves and splits like any packet, it gets the virtual origin
 * position - r dir and a rotation that takes the centre of its level-l pixel
 * pix_v (the descendant or ancestor of the merging pixel p along the first
 * nested sub-pixel) onto the merged direction: the cell's sphere rotation
 * after the shortest rotation from n(l, pix_v) to n(l_merge, p). */

/* The merging sphere of each cell is rotated by a uniform rotation drawn
 * from three uniforms per (step, cell), passed in as inputs (umerge[3 cell]). */

/* Shortest rotation taking unit vector a onto unit vector b (Rodrigues):
 * R = I + [v]x + [v]x^2 / (1 + c), v = a x b, c = a . b (a != -b). */
static void rotation_between(const double a[3], const double b[3], double R[9])
{
    const double v[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    const double c = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    const double K[9] = {0, -v[2], v[1], v[2], 0, -v[0], -v[1], v[0], 0};
    const double f = 1.0 / (1.0 + c);
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double k2 = 0.0;
            for (int m = 0; m < 3; m++) k2 += K[3 * i + m] * K[3 * m + j];
            R[3 * i + j] = (i == j ? 1.0 : 0.0) + K[3 * i + j] + f * k2;
        }
}

static void mat_mul(const double A[9], const double B[9], double C[9])
{
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double v = 0.0;
            for (int m = 0; m < 3; m++) v += A[3 * i + m] * B[3 * m + j];
            C[3 * i + j] = v;
        }
}

typedef struct {
    long long key;           /* cell * 2^20 + merging pixel */
    long long idx;
} merge_key;

static int cmp_desc_double(const void* a, const void* b)
{
    const double x = *(const double*)a, y = *(const double*)b;
    return (x < y) - (x > y);
}

static int cmp_merge_key(const void* a, const void* b)
{
    const merge_key* x = (const merge_key*)a;
    const merge_key* y = (const merge_key*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/* Merge the carried packets in *list (in place: exempt and ungrouped packets
 * keep their order, the merged packets follow in (cell, pixel) order). */
static int merge_carried(const orc_state* S, orc_vec* list, const double* umerge, orc_ledger* L)
{
    const orc_params* P = &S->p;
    const int nb = P->n_bins;
    const long long n = list->n;
    const long long E = (long long)floor(P->merge_exempt * (double)S->ncell);
    if (n == 0 || E >= n) return 0;
    double* ph = (double*)malloc(sizeof(double) * n);
    double* sorted = (double*)malloc(sizeof(double) * n);
    merge_key* keys = (merge_key*)malloc(sizeof(merge_key) * n);
    orc_ray* out = (orc_ray*)malloc(sizeof(orc_ray) * n);
    if (!ph || !sorted || !keys || !out) return -1;
    for (long long j = 0; j < n; j++) ph[j] = sum_bins(list->v[j].N, nb);
    memcpy(sorted, ph, sizeof(double) * n);
    qsort(sorted, n, sizeof(double), cmp_desc_double);
    const double T = E >= 1 ? sorted[E - 1] : INFINITY;
    csum before = {0, 0}, after = {0, 0};
    long long nk = 0, m = 0;
    for (long long j = 0; j < n; j++) {
        csum_add(&before, ph[j]);
        const orc_ray* r = &list->v[j];
        if (ph[j] >= T) continue;
        double pos[3];
        long long c[3];
        for (int a = 0; a < 3; a++) pos[a] = r->origin[a] + r->r * r->dir[a];
        locate(P, pos, r->dir, c);
        const long long cell = c[0] + (long long)P->nx * (c[1] + (long long)P->ny * c[2]);
        double R[9], nloc[3];
        shoemake_rotation(umerge + 3 * cell, R);
        for (int a = 0; a < 3; a++) nloc[a] = R[a] * r->dir[0] + R[3 + a] * r->dir[1] + R[6 + a] * r->dir[2];
        const long long pix = healpix_nest_pixel(P->merge_level, nloc);
        keys[nk].key = cell * (1LL << 20) + pix;
        keys[nk].idx = j;
        nk++;
    }
    qsort(keys, nk, sizeof(merge_key), cmp_merge_key);
    /* the exempt packets and the groups of one keep their place in the list */
    char* keep = (char*)calloc(n, 1);
    if (!keep) return -1;
    for (long long j = 0; j < n; j++) keep[j] = ph[j] >= T;
    for (long long g = 0; g < nk;) {
        long long h = g + 1;
        while (h < nk && keys[h].key == keys[g].key) h++;
        if (h - g == 1) keep[keys[g].idx] = 1;
        g = h;
    }
    m = 0;
    for (long long j = 0; j < n; j++)
        if (keep[j]) out[m++] = list->v[j];
    free(keep);
    for (long long g = 0; g < nk;) {
        long long h = g + 1;
        while (h < nk && keys[h].key == keys[g].key) h++;
        if (h - g >= 2) {
            orc_ray mr;
            memset(&mr, 0, sizeof(mr));
            double W = 0.0, pos[3] = {0, 0, 0}, rsum = 0.0, lsum = 0.0;
            for (long long q = g; q < h; q++) {
                const orc_ray* r = &list->v[keys[q].idx];
                const double w = ph[keys[q].idx];
                W += w;
                for (int a = 0; a < 3; a++) pos[a] += w * (r->origin[a] + r->r * r->dir[a]);
                rsum += w * r->r;
                lsum += w * (double)r->level;
                for (int b = 0; b < nb; b++) mr.N[b] += r->N[b];
            }
            const long long cell = keys[g].key >> 20;
            const long long p = keys[g].key & ((1LL << 20) - 1);
            for (int a = 0; a < 3; a++) pos[a] /= W;
            mr.r = rsum / W;
            mr.r_stop = mr.r;
            mr.level = (int)floor(lsum / W + 0.5);
            const int lm = P->merge_level;
            mr.pix = mr.level >= lm ? p << (2 * (mr.level - lm)) : p >> (2 * (lm - mr.level));
            double Rc[9], nb_m[3], nb_v[3], RA[9];
            shoemake_rotation(umerge + 3 * cell, Rc);
            healpix_nest_center(lm, p, nb_m);
            healpix_nest_center(mr.level, mr.pix, nb_v);
            rotation_between(nb_v, nb_m, RA);
            mat_mul(Rc, RA, mr.R);
            set_direction(&mr);
            for (int a = 0; a < 3; a++) mr.origin[a] = pos[a] - mr.r * mr.dir[a];
            for (int b = 0; b < nb; b++) mr.Ninit[b] = mr.N[b];
            mr.src = -1;
            out[m++] = mr;
            L->merges++;
            L->rays_merged += h - g;
        }
        g = h;
    }
    for (long long j = 0; j < m; j++) csum_add(&after, sum_bins(out[j].N, nb));
    L->merge_residual += csum_get(&before) - csum_get(&after);
    memcpy(list->v, out, sizeof(orc_ray) * m);
    list->n = m;
    free(ph); free(sorted); free(keys); free(out);
    return 0;
}

/* ------------------------------------------------------------ state API */
orc_state* orc_create(const orc_params* P, const float* nH, const float* kappa, const double* x0)
{
    if (!P || P->nx < 1 || P->ny < 1 || P->nz < 1 || P->n_bins < 1 || P->n_bins > ORC_MAX_BINS) return NULL;
    if (P->opacity_mode != 0 && P->opacity_mode != 1) return NULL;
    if (P->temperature && P->opacity_mode == 1 && !(P->t_reion > 0.0)) return NULL;
    orc_state* S = (orc_state*)calloc(1, sizeof(orc_state));
    if (!S) return NULL;
    S->p = *P;
    if (S->p.n_chunks < 1) S->p.n_chunks = 16;
    S->ncell = (long long)P->nx * P->ny * P->nz;
    S->nH = (double*)malloc(sizeof(double) * S->ncell);
    S->kappa = (double*)malloc(sizeof(double) * S->ncell);
    S->x = (double*)malloc(sizeof(double) * S->ncell);
    S->gamma = (double*)calloc(S->ncell, sizeof(double));
    S->T = (double*)malloc(sizeof(double) * S->ncell);
    if (!S->nH || !S->kappa || !S->x || !S->gamma || !S->T) return NULL;
    for (long long i = 0; i < S->ncell; i++) {
        S->nH[i] = nH[i];
        S->kappa[i] = kappa ? kappa[i] : 0.0;
        S->x[i] = x0 ? x0[i] : 1.0;
        S->T[i] = 1e4;
    }
    return S;
}

/* Gas temperature of every cell, K (the state keeps it; it evolves when
 * the temperature is on). */
void orc_set_temperature(orc_state* S, const double* T)
{
    for (long long i = 0; i < S->ncell; i++) S->T[i] = T[i];
}

void orc_read_temperature(const orc_state* S, double* T) { memcpy(T, S->T, sizeof(double) * S->ncell); }

/* New absorption-coefficient field, the rest of the state kept (the caller's
 * opacity model between steps, §4.2 Eq. lambda_nu_general). */
void orc_set_kappa(orc_state* S, const float* kappa)
{
    for (long long i = 0; i < S->ncell; i++) S->kappa[i] = kappa[i];
}

/* New hydrogen density field between steps, the rest of the state kept
 * (the density a simulation hands to the next step).  The temperature takes
 * the compression term of Eq. temp_evolution_standard, dT/dt = (2 T / 3
 * Delta) dDelta/dt, whose solution over any path is T Delta^(-2/3) constant:
 * T -> T (Delta_new / Delta_old)^(2/3) with Delta = n_H / <n_H> over the grid
 * (a change of the mean alone is the Hubble term's); cells with n_H = 0
 * before or after keep T.  Returns -1 if a mean is not > 0. */
int orc_set_density(orc_state* S, const float* nH)
{
    double m0 = 0.0, m1 = 0.0;
    for (long long i = 0; i < S->ncell; i++) {
        m0 += S->nH[i];
        m1 += (double)nH[i];
    }
    if (!(m0 > 0.0) || !(m1 > 0.0)) return -1;
    m0 /= (double)S->ncell;
    m1 /= (double)S->ncell;
    for (long long i = 0; i < S->ncell; i++) {
        const double n1 = (double)nH[i];
        if (S->p.temperature && S->nH[i] > 0.0 && n1 > 0.0) S->T[i] *= pow((n1 / m1) / (S->nH[i] / m0), 2.0 / 3.0);
        S->nH[i] = n1;
    }
    return 0;
}

void orc_destroy(orc_state* S)
{
    if (!S) return;
    free(S->carried.v);
    free(S->nH); free(S->kappa); free(S->x); free(S->gamma); free(S->T);
    free(S->src_pos); free(S->ndot);
    free(S);
}

int orc_set_sources(orc_state* S, int nsrc, const double* pos, const double* ndot)
{
    free(S->carried.v);
    memset(&S->carried, 0, sizeof(S->carried));
    free(S->src_pos); free(S->ndot);
    S->nsrc = nsrc;
    S->src_pos = (double*)malloc(sizeof(double) * 3 * (nsrc > 0 ? nsrc : 1));
    S->ndot = (double*)malloc(sizeof(double) * S->p.n_bins * (nsrc > 0 ? nsrc : 1));
    if (!S->src_pos || !S->ndot) return -1;
    memcpy(S->src_pos, pos, sizeof(double) * 3 * nsrc);
    memcpy(S->ndot, ndot, sizeof(double) * S->p.n_bins * nsrc);
    return 0;
}

/* One step of length dt.  u holds three uniforms per source for this step's
 * sphere rotation.  Order: opacity snapshot, casting, march of every packet
 * (carried and new), chemistry, ledger.  Sources are cut into n_chunks
 * fixed chunks, each with its own Gamma buffer and ledger, summed in chunk
 * order, so the result does not depend on the thread count.
 *
 * With chem_iterations = K >= 1 the step follows the iteration of §4.1:
 * the first march sees n_HI of the start of the step; after march k < K the
 * time-averaged <x> of every cell (Eq. avg_xi, with that march's Gamma and
 * n_e = n_H (1 - <x>) of the previous estimate, first x0) gives the n_HI the
 * next march sees (Eq. gamma_updated_standard).  Each march starts from the
 * same packets, and only the last one's deposits, ledger and carried packets
 * are kept; x(dt) (Eq. xi_of_t) then uses the last Gamma and n_e of the last
 * estimate.
 *
 * In the Generalized Opacity Mode chem_iterations = K >= 1 iterates the
 * ionized gas's opacity with Gamma (§4.2: Eq. lambda_nu_general and Eq.
 * gamma_avg_subgrid updated in turn), with the equilibrium opacity of §5.1:
 * kappa_nu = sigma_nu n_HI (Eq. subgrid_lambda), n_HI from photo-ionization
 * equilibrium, alpha n_H^2 / Gamma (Eqs. equilibrium_condition and
 * subgrid_nHI), at most n_H (no photons: neutral), added to the input kappa.
 * Each march sees n_HI from the Gamma of the march before it, the first
 * march of a step the last Gamma of the previous step (the iteration runs
 * to a self-consistent solution, so its first guess only sets how many
 * marches that takes); where no rate is known yet (no photons so far) the
 * first guess is the optically thin one of Eq. gamma_initial_subgrid
 * (n_HI = 0).  Each march starts from the same packets, and only the last
 * one's deposits, front photons, ledger and carried packets are kept. */
int orc_step(orc_state* S, double dt, const double* u, const double* umerge, int nthreads)
{
    const orc_params* P = &S->p;
    const int nb = P->n_bins;
    const int K = P->n_chunks;
    const long long N = S->ncell;
    double* nHI = (double*)malloc(sizeof(double) * N);
    double* gk = (double*)calloc((size_t)K * N, sizeof(double));
    chunk_ledger* Lk = (chunk_ledger*)calloc(K, sizeof(chunk_ledger));
    orc_vec* new_flight = (orc_vec*)calloc(K, sizeof(orc_vec));   /* per chunk */
    if (!nHI || !gk || !Lk || !new_flight) return -1;
    const int n_iter = P->chem_iterations > 0 ? P->chem_iterations : 1;
    const int gen = P->opacity_mode == 1;
    double* xion = NULL;
    double* fk = NULL;
    double* kap = NULL;   /* the ionized gas's kappa each march sees (Generalized Opacity Mode) */
    if (gen) {
        xion = (double*)malloc(sizeof(double) * N);
        fk = (double*)calloc((size_t)K * N, sizeof(double));
        kap = (double*)malloc(sizeof(double) * N);
        if (!xion || !fk || !kap) return -1;
        for (long long i = 0; i < N; i++) {
            xion[i] = 1.0 - S->x[i];
            kap[i] = S->kappa[i];
        }
    }
    double* hk = NULL;    /* per-chunk photo-heating, eV per cell (temperature on, Standard Mode) */
    if (P->temperature && !gen) {
        hk = (double*)calloc((size_t)K * N, sizeof(double));
        if (!hk) return -1;
    }
    /* the rates of the step, at its starting temperature */
    double* alpha_c = (double*)malloc(sizeof(double) * N);
    double* coll_c = (double*)malloc(sizeof(double) * N);
    if (!alpha_c || !coll_c) return -1;
    for (long long i = 0; i < N; i++) {
        if (P->temperature) {
            double r[7];
            orc_rates(S->T[i], r);
            alpha_c[i] = r[0];
            coll_c[i] = r[1];
        } else {
            alpha_c[i] = P->alpha_B;
            coll_c[i] = P->coll_ion;
        }
    }
    double* xavg = NULL;
    if (P->chem_iterations > 0 && !gen) {
        xavg = (double*)malloc(sizeof(double) * N);
        if (!xavg) return -1;
        memcpy(xavg, S->x, sizeof(double) * N);
    }
    const double V = P->dx * P->dx * P->dx;
    const long long ncast = 12LL << (2 * P->base_level);
    if (nthreads < 1) nthreads = 1;

    for (int it = 0; it < n_iter; it++) {
        for (long long i = 0; i < N; i++) nHI[i] = S->nH[i] * (xavg ? xavg[i] : S->x[i]);
        if (gen && P->chem_iterations > 0)
            for (long long i = 0; i < N; i++) {
                /* equilibrium n_HI of the ionized gas from the last march's
                 * Gamma (the previous step's at the first march), with
                 * alpha_B at the step's starting temperature when it
                 * evolves; where no rate is known yet the optically thin
                 * guess */
                const double nH = S->nH[i], g = S->gamma[i];
                double nhi = 0.0;
                if (g > 0.0) nhi = (alpha_c[i] * nH * nH < g * nH) ? alpha_c[i] * nH * nH / g : nH;
                kap[i] = S->kappa[i] + P->sigma[0] * nhi;
            }
        if (it > 0) {
            /* the march starts again from the step's packets */
            memset(gk, 0, sizeof(double) * (size_t)K * N);
            if (gen) memset(fk, 0, sizeof(double) * (size_t)K * N);
            if (hk) memset(hk, 0, sizeof(double) * (size_t)K * N);
            memset(Lk, 0, sizeof(chunk_ledger) * K);
            for (int k = 0; k < K; k++) {
                free(new_flight[k].v);
                memset(&new_flight[k], 0, sizeof(orc_vec));
            }
        }

#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
        for (int k = 0; k < K; k++) {
            orc_vec stack = {0, 0, 0};
            march_ctx M;
            M.S = S; M.nHI = nHI; M.gamma = gk + (size_t)k * N; M.L = Lk + k;
            M.stack = &stack; M.inv_vdt = 1.0 / (V * dt);
            M.xion = xion; M.front = gen ? fk + (size_t)k * N : NULL; M.kappa = kap;
            M.heat = hk ? hk + (size_t)k * N : NULL;
            M.flight_out = &new_flight[k];
            /* packets carried from the previous step get a fresh budget */
            const long long nc = S->carried.n;
            for (long long j = nc * k / K; j < nc * (k + 1) / K; j++) {
                orc_ray ray = S->carried.v[j];
                ray.r_stop = ray.r + P->c_ray * dt;
                march_one_ray(&M, &ray);
                drain(&M);
            }
            int s0 = (int)(((long long)S->nsrc * k) / K), s1 = (int)(((long long)S->nsrc * (k + 1)) / K);
            for (int s = s0; s < s1; s++) {
                /* casting on this step's rotated sphere (§3.1, Eq. Nray) */
                double R[9];
                shoemake_rotation(u + 3 * s, R);
                for (long long p = 0; p < ncast; p++) {
                    orc_ray ray;
                    memset(&ray, 0, sizeof(ray));
                    ray.src = s; ray.level = P->base_level; ray.pix = p;
                    memcpy(ray.R, R, sizeof(R));
                    for (int a = 0; a < 3; a++) ray.origin[a] = S->src_pos[3 * s + a];
                    set_direction(&ray);
                    ray.r = 0.0;
                    ray.r_stop = P->c_ray * dt;
                    for (int b = 0; b < nb; b++) {
                        ray.N[b] = S->ndot[(size_t)s * nb + b] * dt / (double)ncast;
                        ray.Ninit[b] = ray.N[b];
                        csum_add(&M.L->emitted, ray.N[b]);
                    }
                    M.L->rays_emitted++;
                    march_one_ray(&M, &ray);
                    drain(&M);
                }
            }
            free(stack.v);
        }

        /* deterministic chunk-ordered reduction */
        for (long long i = 0; i < N; i++) {
            double g = 0.0;
            for (int k = 0; k < K; k++) g += gk[(size_t)k * N + i];
            S->gamma[i] = g;
        }
        if (it + 1 < n_iter && !gen)
            for (long long i = 0; i < N; i++) {
                double xe;
                const double ne = S->nH[i] * (1.0 - xavg[i]);
                xavg[i] = chemistry_avg(S->x[i], S->gamma[i], ne, alpha_c[i], coll_c[i], dt, &xe);
            }
    }

    long long cross = 0;
    csum tot[6];
    {
        const double prev[6] = {S->L.emitted, S->L.absorbed_HI, S->L.absorbed_sub, S->L.escaped, S->L.dropped,
                                S->L.absorbed_front};
        for (int j = 0; j < 6; j++) { tot[j].s = prev[j]; tot[j].c = 0.0; }
    }
    for (int k = 0; k < K; k++) {
        csum_add(&tot[0], csum_get(&Lk[k].emitted));
        csum_add(&tot[1], csum_get(&Lk[k].absorbed_HI));
        csum_add(&tot[2], csum_get(&Lk[k].absorbed_sub));
        csum_add(&tot[3], csum_get(&Lk[k].escaped));
        csum_add(&tot[4], csum_get(&Lk[k].dropped));
        csum_add(&tot[5], csum_get(&Lk[k].front));
        S->L.crossings += Lk[k].crossings;
        S->L.rays_emitted += Lk[k].rays_emitted;
        S->L.splits += Lk[k].splits;
        S->L.n_escaped += Lk[k].n_escaped;
        S->L.n_dropped += Lk[k].n_dropped;
        cross += Lk[k].crossings;
    }
    S->L.emitted = csum_get(&tot[0]);
    S->L.absorbed_HI = csum_get(&tot[1]);
    S->L.absorbed_sub = csum_get(&tot[2]);
    S->L.escaped = csum_get(&tot[3]);
    S->L.dropped = csum_get(&tot[4]);
    S->L.absorbed_front = csum_get(&tot[5]);
    S->last_crossings = cross;

    /* carried packets replace the old list, in chunk order, then merge */
    orc_vec list = {0, 0, 0};
    for (int k = 0; k < K; k++)
        for (long long j = 0; j < new_flight[k].n; j++)
            if (vec_push(&list, &new_flight[k].v[j])) return -1;
    for (int k = 0; k < K; k++) free(new_flight[k].v);
    if (P->merge && umerge && merge_carried(S, &list, umerge, &S->L)) return -1;
    free(S->carried.v);
    S->carried = list;
    csum inflight = {0.0, 0.0};
    for (long long j = 0; j < list.n; j++) csum_add(&inflight, sum_bins(list.v[j].N, nb));
    S->L.in_flight = csum_get(&inflight);
    S->L.n_in_flight = list.n;

    /* chemistry closes the step */
    if (gen) {
        /* moving screen (§4.2, Eq. dxidt): the photons stopped at a cell's
         * front ionize (1 + chi) atoms each; the ionized fraction is at most
         * 1 and no recombination moves the front back.  Photons beyond the
         * atoms the cell had left ionize nothing: they move from
         * absorbed_front to front_excess */
        csum excess = {0.0, 0.0};
        for (long long i = 0; i < N; i++) {
            double f = 0.0;
            for (int k = 0; k < K; k++) f += fk[(size_t)k * N + i];
            const double atoms = (1.0 + P->he_chi) * S->nH[i] * V;
            double xi;
            if (atoms > 0.0) {
                xi = xion[i] + f / atoms;
                if (xi > 1.0) {
                    const double left = (1.0 - xion[i]) * atoms;
                    if (f > left) csum_add(&excess, f - left);
                    xi = 1.0;
                }
            } else {
                if (f > 0.0) csum_add(&excess, f);   /* no hydrogen: nothing to ionize */
                xi = 1.0;
            }
            S->x[i] = 1.0 - xi;
            if (P->temperature) S->T[i] = mixed_temperature(P, S->T[i], S->nH[i], S->gamma[i], xion[i], xi, dt);
        }
        const double ex = csum_get(&excess);
        S->L.absorbed_front -= ex;
        S->L.front_excess += ex;
        free(xion); free(fk); free(kap);
    } else {
        /* the hydrogen update, then (temperature on) the temperature from
         * the step's photo-heating with the new neutral fraction */
        csum heat_in = {S->L.heat_in, 0.0};
        for (long long i = 0; i < N; i++) {
            const double x0 = S->x[i];
            if (xavg) {
                double xe;
                const double ne = S->nH[i] * (1.0 - xavg[i]);
                (void)chemistry_avg(x0, S->gamma[i], ne, alpha_c[i], coll_c[i], dt, &xe);
                S->x[i] = xe;
            } else {
                S->x[i] = chemistry_be(x0, S->gamma[i], S->nH[i], alpha_c[i], coll_c[i], dt);
            }
            if (hk) {
                double e = 0.0;
                for (int k = 0; k < K; k++) e += hk[(size_t)k * N + i];
                csum_add(&heat_in, e * ORC_EV);
                S->T[i] = temperature_update(P, S->T[i], S->nH[i], x0, S->x[i], e * ORC_EV / (V * dt), dt);
            }
        }
        S->L.heat_in = csum_get(&heat_in);
        free(xavg);
    }

    S->step++;
    free(hk); free(alpha_c); free(coll_c);
    free(nHI); free(gk); free(Lk); free(new_flight);
    return 0;
}

/* Per-bin transmitted photons of one ray through the current field (no
 * floor, no cap, no split), for the exact exp(-tau) test. */
int orc_debug_transmit(orc_state* S, const double o[3], const double d[3], const double* N, double dt,
                       double* gamma_out, double* N_exit, double* heat_out)
{
    const orc_params* P = &S->p;
    if (P->opacity_mode != 0) return -1;   /* Standard Mode only */
    orc_state T = *S;
    T.p.max_level = 0;
    T.p.base_level = 0;
    T.p.flux_floor = 0.0;
    T.p.max_dist = 0.0;
    double src[3] = {o[0], o[1], o[2]};
    T.src_pos = src;
    T.nsrc = 1;
    double* nHI = (double*)malloc(sizeof(double) * S->ncell);
    if (!nHI) return -1;
    for (long long i = 0; i < S->ncell; i++) nHI[i] = S->nH[i] * S->x[i];
    orc_vec stack = {0, 0, 0}, fl = {0, 0, 0};
    chunk_ledger L;
    memset(&L, 0, sizeof(L));
    march_ctx M;
    M.S = &T; M.nHI = nHI; M.gamma = gamma_out; M.L = &L; M.stack = &stack; M.flight_out = &fl;
    M.inv_vdt = 1.0 / (P->dx * P->dx * P->dx * dt);
    M.xion = NULL; M.front = NULL; M.kappa = NULL; M.heat = heat_out;
    orc_ray ray;
    memset(&ray, 0, sizeof(ray));
    for (int a = 0; a < 3; a++) {
        ray.dir[a] = d[a];
        ray.origin[a] = o[a];
    }
    ray.r = 0.0; ray.r_stop = INFINITY;
    for (int b = 0; b < P->n_bins; b++) { ray.N[b] = N[b]; ray.Ninit[b] = N[b]; }
    /* march with the exit photons captured per bin */
    orc_vec out = {0, 0, 0};
    M.flight_out = &out;
    march_one_ray(&M, &ray);
    /* the ray object holds the photons it carried when it stopped */
    for (int b = 0; b < P->n_bins; b++) N_exit[b] = ray.N[b];
    free(stack.v); free(fl.v); free(out.v); free(nHI);
    return (int)L.crossings;
}

/* ------------------------------------------------------------- readout */
void orc_read(const orc_state* S, double* x, double* gamma)
{
    if (x) memcpy(x, S->x, sizeof(double) * S->ncell);
    if (gamma) memcpy(gamma, S->gamma, sizeof(double) * S->ncell);
}

/* Distances from their sources (cm) of the packets carried into the next
 * step, in source order; returns how many there are (at most cap written). */
long long orc_flight_radii(const orc_state* S, double* out, long long cap)
{
    for (long long j = 0; j < S->carried.n && j < cap; j++) out[j] = S->carried.v[j].r;
    return S->carried.n;
}

/* The carried packets, one row of 9 + n_bins doubles each: r, origin (3),
 * direction (3), level, pixel, photons per bin; returns how many there are
 * (rows written up to cap). */
long long orc_flight_dump(const orc_state* S, double* out, long long cap)
{
    const int w = 9 + S->p.n_bins;
    for (long long j = 0; j < S->carried.n && j < cap; j++) {
        const orc_ray* r = &S->carried.v[j];
        double* o = out + j * w;
        o[0] = r->r;
        for (int a = 0; a < 3; a++) {
            o[1 + a] = r->origin[a];
            o[4 + a] = r->dir[a];
        }
        o[7] = r->level;
        o[8] = (double)r->pix;
        for (int b = 0; b < S->p.n_bins; b++) o[9 + b] = r->N[b];
    }
    return S->carried.n;
}

/* Merge the carried packets now, as the end of a step does (for tests: a
 * step run without merging, then this). */
int orc_merge_now(orc_state* S, const double* umerge)
{
    const double before = S->L.in_flight;
    if (merge_carried(S, &S->carried, umerge, &S->L)) return -1;
    csum inflight = {0.0, 0.0};
    for (long long j = 0; j < S->carried.n; j++) csum_add(&inflight, sum_bins(S->carried.v[j].N, S->p.n_bins));
    S->L.in_flight = csum_get(&inflight);
    S->L.n_in_flight = S->carried.n;
    (void)before;
    return 0;
}

/* Backward-Euler update of a whole field (chemistry_be per cell): x_out[i]
 * from x[i], gamma[i], nH[i]. */
void orc_chemistry_field(long long n, const double* x, const double* gamma, const double* nH, double alpha,
                         double coll, double dt, double* x_out)
{
    for (long long i = 0; i < n; i++) x_out[i] = chemistry_be(x[i], gamma[i], nH[i], alpha, coll, dt);
}

void orc_ledger_get(const orc_state* S, orc_ledger* L) { *L = S->L; }
long long orc_last_crossings(const orc_state* S) { return S->last_crossings; }
long long orc_step_index(const orc_state* S) { return S->step; }

/* Checkpoint: neutral fraction, the last step's rate (the first guess of
 * the equilibrium iteration of the Generalized Opacity Mode), temperature,
 * carried packets, ledger, step index. */
long long orc_state_bytes(const orc_state* S)
{
    return (long long)(sizeof(long long) * 3 + sizeof(orc_ledger) + 3 * sizeof(double) * S->ncell +
                       sizeof(orc_ray) * S->carried.n);
}

int orc_save(const orc_state* S, unsigned char* buf)
{
    unsigned char* p = buf;
    long long hdr[2] = {S->step, S->nsrc};
    memcpy(p, hdr, sizeof(hdr)); p += sizeof(hdr);
    memcpy(p, &S->L, sizeof(orc_ledger)); p += sizeof(orc_ledger);
    memcpy(p, S->x, sizeof(double) * S->ncell); p += sizeof(double) * S->ncell;
    memcpy(p, S->gamma, sizeof(double) * S->ncell); p += sizeof(double) * S->ncell;
    memcpy(p, S->T, sizeof(double) * S->ncell); p += sizeof(double) * S->ncell;
    long long n = S->carried.n;
    memcpy(p, &n, sizeof(n)); p += sizeof(n);
    if (n > 0) memcpy(p, S->carried.v, sizeof(orc_ray) * n);
    return 0;
}

int orc_load(orc_state* S, const unsigned char* buf)
{
    const unsigned char* p = buf;
    long long hdr[2];
    memcpy(hdr, p, sizeof(hdr)); p += sizeof(hdr);
    if (hdr[1] != S->nsrc) return -1;
    S->step = hdr[0];
    memcpy(&S->L, p, sizeof(orc_ledger)); p += sizeof(orc_ledger);
    memcpy(S->x, p, sizeof(double) * S->ncell); p += sizeof(double) * S->ncell;
    memcpy(S->gamma, p, sizeof(double) * S->ncell); p += sizeof(double) * S->ncell;
    memcpy(S->T, p, sizeof(double) * S->ncell); p += sizeof(double) * S->ncell;
    long long n;
    memcpy(&n, p, sizeof(n)); p += sizeof(n);
    free(S->carried.v);
    memset(&S->carried, 0, sizeof(S->carried));
    for (long long j = 0; j < n; j++) {
        orc_ray r;
        memcpy(&r, p, sizeof(r)); p += sizeof(r);
        if (vec_push(&S->carried, &r)) return -1;
    }
    return 0;
}

int orc_sizeof_ray(void) { return (int)sizeof(orc_ray); }
int orc_sizeof_ledger(void) { return (int)sizeof(orc_ledger); }
int orc_sizeof_params(void) { return (int)sizeof(orc_params); }
