/*
 * HWFV1 CPU oracle: a plain, slow, single-threaded FP64 implementation of the
 * Haar-wavelet adaptive first-order finite-volume shallow-water timestep
 * (Chowdhury, Kesserwani, Rouge, Richmond, "GPU-parallelisation of
 * wavelet-based grid adaptation for fast finite volume modelling", 2022).
 *
 * THIS IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  The product path (the HIP
 * library under paper_2206_05761_amd/) never calls, links or includes it, and
 * the two share no code.
 *
 * Layout used inside the oracle: one plain row-major array per refinement
 * level n (side 2^n, element [j * 2^n + i], i = column / x, j = row / y).
 * Getters that hand data to tests convert to the Z-order hierarchy index of
 * Section 2.2.1 (Morton code within a level, levels concatenated coarse to
 * fine) with the oracle's own Morton routine.
 *
 * Parity pins: every function here is checked by the CPU tests against
 * worked examples printed in the paper (Fig. 5 Morton table, footnote 2 index
 * example, the L = 2 traversal example of Sections 2.1.2 and 2.2.2), closed
 * forms (Haar round trip, linear ramp, friction recursion, rain), invariants
 * (lake at rest, mass with closed walls, eps = 0 equals uniform FV1,
 * checkpoint/resume) and the exact 1D dam-break Riemann solution.
 */
#ifndef HWFV1_ORACLE_H
#define HWFV1_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_MAX_L 14

enum { OR_BC_WALL = 0, OR_BC_OPEN = 1 };
enum { OR_W = 0, OR_E = 1, OR_S = 2, OR_N = 3 };

/* Problem definition: the user inputs L, eps, t_end of Algorithm 3 plus the
 * physical constants and forcing of Eq. 1. */
typedef struct oracle_problem {
    int32_t L;            /* finest refinement level, grid 2^L x 2^L      */
    int32_t bc[4];        /* W, E, S, N: OR_BC_WALL or OR_BC_OPEN          */
    double eps;           /* error threshold epsilon >= 0                  */
    double g;             /* gravitational acceleration (m/s^2)            */
    double cfl;           /* CFL number (0.5)                              */
    double h_tol;         /* wet/dry depth threshold (m)                   */
    double dx, dy;        /* finest cell size (m)                          */
    double dt_max;        /* largest timestep; also used when all is dry   */
    double manning_n;     /* Manning coefficient n_M (s m^-1/3), 0 = none  */
    double rain_rate;     /* uniform rainfall (m/s)                        */
    double inlet_y0, inlet_y1;     /* west-edge inflow segment (m)        */
    double q_peak, t_peak, t_base; /* triangular hydrograph (m^3/s, s, s) */
    double t_end;         /* simulation end time (s); +inf for none        */
    double zsmax;         /* s_max of the bed when > 0 (the largest bed
                             coefficient of the domain's own finest cells,
                             for a domain padded to the square grid); 0:
                             max(1, max |z|) over the grid                 */
} oracle_problem;

typedef struct oracle_state oracle_state;

/* Scalars returned by oracle_get_scalars, in this order. */
enum {
    OR_SC_T = 0, OR_SC_DT, OR_SC_STEP, OR_SC_NLEAVES, OR_SC_MASS,
    OR_SC_CLIPS, OR_SC_MAXSPEED, OR_SC_LEAF_UPDATES,
    OR_SC_SMAX_H, OR_SC_SMAX_QX, OR_SC_SMAX_QY, OR_SC_SMAX_Z, OR_SC_COUNT
};

/* Create from row-major finest-grid inputs (4^L values each).  Performs the
 * initial discretisation of Algorithm 3 (first line inside the algorithm):
 * stores s^(L), encodes the static bed, flags its significant details and
 * computes the first timestep.  Returns NULL on invalid input. */
oracle_state* oracle_create(const oracle_problem* p, const double* h,
                            const double* qx, const double* qy,
                            const double* z);
void oracle_destroy(oracle_state* st);

/* Restart support: overwrite t, dt and the step counter. */
void oracle_set_time(oracle_state* st, double t, double dt, int64_t step);

/* The phases of one timestep (Algorithm 3, loop body).  oracle_step runs all
 * of them; the phase functions exist so tests can compare phase by phase. */
void oracle_phase_encode(oracle_state* st);     /* Alg. 1 on h, qx, qy   */
void oracle_phase_regularise(oracle_state* st); /* neighbour refinement  */
void oracle_phase_traverse(oracle_state* st);   /* Alg. 2 leaf list      */
void oracle_phase_fv1(oracle_state* st);        /* FV1 update, t, dt     */
int  oracle_step(oracle_state* st);             /* 1 if a step was taken */
int64_t oracle_run(oracle_state* st, int64_t max_steps);

/* Uniform-grid FV1 step on the finest grid (the eps = 0 special case). */
void oracle_uniform_fv1_step(oracle_state* st);

/* Getters.  var: 0 = h, 1 = qx, 2 = qy, 3 = z. */
void oracle_get_fine(const oracle_state* st, double* h, double* qx,
                     double* qy);                   /* row-major          */
void oracle_get_hierarchy(const oracle_state* st, int var, double* out);
                                 /* Z-order index layout, levels 0..L     */
void oracle_get_details(const oracle_state* st, int var, double* out);
                                 /* [3][(4^L-1)/3]: d_alpha, d_beta,
                                    d_gamma in Z-order index layout       */
void oracle_get_flags(const oracle_state* st, int which, uint8_t* out);
                                 /* which: 0 raw (incl. bed), 1 sig after
                                    regularisation, 2 static bed flags;
                                    (4^L-1)/3 bytes, Z-order index layout */
int64_t oracle_get_leaves(const oracle_state* st, uint32_t* idx);
                                 /* hierarchy Z-order indices, DFT order  */
void oracle_get_scalars(const oracle_state* st, double* out);

/* Building blocks exposed for unit pins. */
uint32_t oracle_morton(uint32_t i, uint32_t j);
uint64_t oracle_zindex(int n, uint32_t i, uint32_t j);
void oracle_haar_encode(const double s[4], double out[4]); /* s,da,db,dg */
void oracle_haar_decode(const double c[4], double out[4]); /* s0..s3     */
/* Whole-field round trip: encode row-major finest field f to all levels,
 * then decode level by level from the root with the stored details. */
void oracle_roundtrip(int L, const double* f, double* out);
/* One x-direction face: left state, right state -> flux (mass, normal
 * momentum, tangential momentum) and the two reconstructed depths. */
void oracle_face_flux(const oracle_problem* p, const double left[4],
                      const double right[4], double flux[3],
                      double hstar[2]);
/* Algorithm 2 on a given significance array (Z-order index layout,
 * (4^L-1)/3 bytes): writes the leaf indices in DFT order, returns count. */
int64_t oracle_dft_from_flags(int L, const uint8_t* sig, uint32_t* leaves);
/* Regularisation on a given raw flag array (Z-order index layout). */
void oracle_regularise_flags(int L, const uint8_t* raw, uint8_t* sig);

#ifdef __cplusplus
}
#endif
#endif
