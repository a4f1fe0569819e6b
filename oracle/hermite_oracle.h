/*
 * C interface of the FP64 CPU oracle (test infrastructure only; see
 * hermite_oracle.c).  Not used by, and not shared with, the GPU library.
 */
#ifndef HERMITE_ORACLE_H
#define HERMITE_ORACLE_H
#include <stdint.h>

enum { HWO_PERIODIC = 0, HWO_DIRICHLET = 1, HWO_NEUMANN = 2 };
enum { HWO_DISS_FULL = 0, HWO_DISS_SIMPLE = 1, HWO_CONSERVATIVE = 2 };
enum { HWO_PRIMAL = 0, HWO_DUAL = 1 };

typedef struct {
    int d;             /* space dimension, 1..3 */
    int m;             /* nodal degree */
    int n[3];          /* cells per dimension */
    double xl[3], xr[3];
    double c, dt;
    int bc[3];         /* HWO_PERIODIC / HWO_DIRICHLET / HWO_NEUMANN */
    int method;        /* HWO_DISS_FULL / HWO_DISS_SIMPLE / HWO_CONSERVATIVE */
    int taylor_stages; /* 0: run the Taylor series until it terminates; >0: truncate */
} hwo_problem;

int hwo_hermite_matrix(int m, double *H);
int64_t hwo_nodes(const hwo_problem *p, int grid);
int hwo_diss_half(const hwo_problem *p, int to_grid, const double *u_in, const double *v_in,
                  double *u_out, double *v_out, const int64_t *sel, int64_t nsel, int nthreads);
/* The same with a forcing term f (u_tt = c^2 Laplacian u + f): f_coef holds, for every */
/* node of the grid written, n_orders blocks of (2m)^d values phi[r][k] =               */
/* h^k/k! d^k/dx^k d^r/dt^r f at that node and the start of the half step.              */
int hwo_diss_half_forced(const hwo_problem *p, int to_grid, const double *u_in, const double *v_in,
                         const double *f_coef, int n_orders, double *u_out, double *v_out,
                         const int64_t *sel, int64_t nsel, int nthreads);
int hwo_cons_half(const hwo_problem *p, int to_grid, const double *u_from, const double *u_old,
                  double *u_new, const int64_t *sel, int64_t nsel, int nthreads);
/* Half steps with forcing and inhomogeneous / time-dependent wall data (Sec. 3.1.3).    */
/* wall_u, wall_v: NULL (homogeneous walls) or the wall records of every face (layout in  */
/* hermite_oracle.c), used on half steps onto the primal grid.  Conservative forcing:     */
/* n_orders blocks of (2m+2)^d values per output node, phi[q][k] = h^k/k! d^k d^q/dt^q f  */
/* at the node and the time of the input level.                                          */
int hwo_diss_half_ext(const hwo_problem *p, int to_grid, const double *u_in, const double *v_in,
                      const double *f_coef, int n_orders, const double *wall_u, const double *wall_v,
                      double *u_out, double *v_out, const int64_t *sel, int64_t nsel, int nthreads);
int hwo_cons_half_ext(const hwo_problem *p, int to_grid, const double *u_from, const double *u_old,
                      const double *f_coef, int n_orders, const double *wall_u, double *u_new,
                      const int64_t *sel, int64_t nsel, int nthreads);
int hwo_cons_startup(const hwo_problem *p, const double *u0, const double *v0, double *u_half,
                     int nthreads);
double hwo_cons_energy(const hwo_problem *p, int grid_a, const double *u_a, const double *u_b_new,
                       const double *u_b_old, int nthreads);
double hwo_seminorm(const hwo_problem *p, int data_grid, const double *f, const double *g,
                    int mdata, int q, int nthreads);
double hwo_diss_energy(const hwo_problem *p, int data_grid, const double *u, const double *v,
                       int nthreads);
#endif
