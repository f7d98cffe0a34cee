/* FP64 CPU oracle of the Kalman-filter track builder and fitter (barrel
 * cylinders and endcap disks).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke check and
 * the benchmark's CPU-baseline leg may call it.  It shares no source, header,
 * table or helper with the GPU library, and the GPU library never calls it.
 *
 * Units: cm, GeV, tesla, radians; field along +z.  A state is
 * (x, y, z, q/pT, phi, theta): global Cartesian position and polar momentum
 * (the paper's hybrid coordinate system, Section 2.2).  Covariances cross this
 * interface packed as the 21-entry upper triangle, row-major.
 */
#ifndef MKF_ORACLE_H
#define MKF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_LAYERS 16
#define ORC_MAX_CANDS 16
#define ORC_MAX_ALT 4
#define ORC_CUT_CONSIDER 0.1      /* |chi2 - cut| below which a decision is re-run */
#define ORC_RANK_CONSIDER 0.01    /* relative key gap below which a rank decision is re-run */

typedef struct {
    int32_t n_layers;
    int32_t n_seed_layers;      /* seeds sit on layer n_seed_layers-1 */
    int32_t max_cands;          /* beam width k */
    int32_t max_holes;
    int32_t hole_always;        /* 1: a hole child even when hits were accepted */
    int32_t update3d;           /* 1: 3x3 global-Cartesian measurement (orc_update_3d) on every layer */
    double radius[ORC_MAX_LAYERS];
    double x0[ORC_MAX_LAYERS];  /* material per layer, radiation lengths at normal incidence */
    double bz;
    double sigma_rphi;
    double sigma_z;
    double chi2_cut;
    double mass;                /* mass hypothesis for the scattering angle */
    int32_t kind[ORC_MAX_LAYERS];   /* 0 cylinder of radius radius[L], 1 disk: plane z = zplane[L] */
    double zplane[ORC_MAX_LAYERS];
    double sigma_r;             /* disk hit resolution along r */
    double thick[ORC_MAX_LAYERS];   /* > 0: hits spread over this radial (cylinder) or z (disk) depth
                                       around the average surface; two-step propagation */
} orc_config;

typedef struct {
    int32_t n_layers;
    int32_t pad_;
    const int32_t *n_hits;      /* [n_layers] */
    const double *const *xyz;   /* [n_layers] -> [n_hits[L]][3] */
} orc_hits;

/* Result of one seed's build (rank-0 candidate after the last layer). */
typedef struct {
    double par[6];
    double cov[21];
    double chi2;
    int32_t hits[ORC_MAX_LAYERS];
    int32_t n_hits;
    int32_t n_holes;
    int32_t status;             /* 0 reached last layer, 1 hole limit, 2 propagation failed */
    int32_t n_final;            /* candidates alive in the final beam */
    /* Decision margins, for the tie protocol of the parity tests.  A
     * decision is relevant when taking it the other way changes the output
     * (the rank-0 hit list or status): every decision within ORC_CUT_CONSIDER
     * of the cut or ORC_RANK_CONSIDER of a rank tie is re-run from the beam
     * before its layer with the decision inverted.  m_cut and m_rank are the
     * smallest margins of relevant decisions and of decisions beyond those
     * windows (not examined); the _raw values count every decision. */
    double m_cut;               /* |chi2 - cut| */
    double m_rank;              /* relative key gap at the k/(k+1) boundary or the final rank-0/rank-1 choice */
    double m_prop;              /* min |distance to tangency| / r over propagations */
    double m_cut_raw;
    double m_rank_raw;
    /* outcomes of the relevant decisions of smallest margin, taken the other
     * way (alt_kind 0 cut, 1 beam boundary, 2 final choice); n_alt of them */
    int32_t n_alt;
    int32_t alt_kind[ORC_MAX_ALT];
    double alt_margin[ORC_MAX_ALT];
    int32_t alt_hits[ORC_MAX_ALT][ORC_MAX_LAYERS];
    int32_t alt_status[ORC_MAX_ALT];
    /* counters */
    int64_t n_prop;             /* candidate-layers propagated */
    int64_t n_accept;           /* (candidate, hit) pairs passing the cut */
    int64_t n_update;           /* KF updates of surviving hit children */
} orc_track;

/* Propagate a state to the cylinder of radius r (closed-form circle
 * intersection).  F (6x6 row-major, may be NULL) receives d(out)/d(in) on the
 * cylinder.  Returns 0 on success, 1 if the helix never reaches r.
 * *margin (may be NULL) receives the signed distance to tangency. */
int orc_propagate(const double par[6], double r, double bz, double out[6],
                  double F[36], double *path, double *margin);

/* Propagate a state to the plane z = zd.  Returns 1 if the helix moves away
 * from it; *margin receives the signed transverse path. */
int orc_propagate_plane(const double par[6], double zd, double bz, double out[6],
                        double F[36], double *path, double *margin);

/* The nearest crossing (either direction) of the cylinder r = where (kind
 * 0) or the plane z = where (kind 1): the second, short step of the two-step
 * propagation.  Returns 1 when the helix never reaches it. */
int orc_step_near(const double par[6], int kind, double where, double bz, double out[6], double F[36],
                  double *path);

/* Add multiple-scattering noise for crossing a layer (kind 0 cylinder, 1
 * disk) of thickness x0 at the state's position (full 6x6 row-major
 * covariance, in place). */
void orc_add_ms(const double par[6], int kind, double x0, double mass, double C[36]);

/* chi2 of a hit against a predicted state (full 6x6 covariance); kind 0
 * measures (r*phi, z), kind 1 (r*phi, r); s2 is the second coordinate's
 * resolution. */
double orc_chi2(const double par[6], const double C[36], const double hit[3], int kind,
                double sigma_rphi, double s2);

/* KF update with one hit; writes the filtered state and covariance and
 * returns the hit's chi2. */
double orc_update(const double par[6], const double C[36], const double hit[3], int kind,
                  double sigma_rphi, double s2, double out_par[6], double out_C[36]);

/* The 3x3 global-Cartesian measurement: the hit's (x, y, z) with error
 * ellipsoid sigma_rphi (along the layer), sigma_r (radial), sigma_z (along z),
 * all positive.  chi2, and the update writing the filtered state. */
double orc_chi2_3d(const double par[6], const double C[36], const double hit[3], double sigma_rphi,
                   double sigma_r, double sigma_z);
double orc_update_3d(const double par[6], const double C[36], const double hit[3], double sigma_rphi,
                     double sigma_r, double sigma_z, double out_par[6], double out_C[36]);

/* Transport C <- F C F^T (full 6x6). */
void orc_transport(const double F[36], double C[36]);

/* Forward fit with known hits (-1 = no hit on that layer).  init_* are the
 * prior at layer 0, packed covariance.  Output: state after the last update,
 * chi2 summed over all updates, ndof = 2*n_updates - 5, status as above.
 * hit_chi2 (may be NULL): [n][n_layers] per-hit chi2 (-1 where no update). */
void orc_fit(const orc_config *cfg, const orc_hits *hits, int32_t n_tracks,
             const double *init_par, const double *init_cov, const int32_t *track_hits,
             double *out_par, double *out_cov, double *out_chi2, int32_t *out_ndof,
             int32_t *out_status, double *hit_chi2, int32_t n_threads);

/* Prior for the final fit of a built track (Section 2: a fit over the hits of
 * a complete track), from its hits on layers 0, 1 and 2: the helix through
 * them - the circle through the three transverse points, z linear in the arc
 * length - evaluated at the first hit, with the covariance
 * diag(sig[0..4])^2 in the frame (u, z, q/pT, phi, theta), u along the layer
 * tangent at the hit's azimuth (on a disk: (u, r, q/pT, phi, theta)).  out_ok[i] = 0 when a hit is missing or the
 * three points are collinear (then out_par/out_cov are zero). */
void orc_circle_prior(const orc_config *cfg, const orc_hits *hits, int32_t n_tracks,
                      const int32_t *track_hits, const double sig[5], double *out_par, double *out_cov,
                      int32_t *out_ok);

/* Combinatorial KF building of the listed seeds (all if seed_ids == NULL).
 * Output row i belongs to seed_ids[i]. */
void orc_build(const orc_config *cfg, const orc_hits *hits, int32_t n_seeds_total,
               const double *seed_par, const double *seed_cov, const int32_t *seed_hits,
               const int32_t *seed_ids, int32_t n_sel, orc_track *out, int32_t n_threads);

/* As orc_build, and also every rank of each seed's final beam:
 * beam[i * max_cands + r] is rank r of seed seed_ids[i] (par, cov, chi2,
 * hits, n_hits, n_holes, status; status -1 for ranks beyond the beam). */
void orc_build_beam(const orc_config *cfg, const orc_hits *hits, int32_t n_seeds_total,
                    const double *seed_par, const double *seed_cov, const int32_t *seed_hits,
                    const int32_t *seed_ids, int32_t n_sel, orc_track *out, orc_track *beam, int32_t n_threads);

/* Replay a given hit list for one seed through the building rules: propagate
 * layer by layer, update with the listed hit (or take a hole for -1).  Writes
 * per-layer chi2 (-1 for holes) and returns the summed chi2; *ok is 0 when a
 * listed hit fails the cut or propagation fails. */
double orc_replay(const orc_config *cfg, const orc_hits *hits, const double seed_par[6],
                  const double seed_cov[21], const int32_t *layer_hits, double *layer_chi2,
                  int32_t *ok);

#ifdef __cplusplus
}
#endif
#endif
