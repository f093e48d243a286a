/*
 * hctm_serve.h -- serving many CTMRG environment solves on one GPU.
 *
 * A server takes independent solves (a tensor, its sizes, chi, the form, a
 * convergence tolerance and an iteration cap) as they arrive and runs them
 * concurrently on a fixed pool of max_active host worker threads, each with
 * its own HIP stream; each admitted solve gets a workspace carved from one
 * device pool allocated when the server is created.  Admission is first come, first served, by memory:
 * the oldest waiting solve starts as soon as its workspace (ctm_workspace_size)
 * fits into the free part of the pool and fewer than max_active solves run.
 * While it runs, its kernels overlap on the device with those of the others.
 *
 * A solve is one ctm_init and then ctm_step(1) until ctm_converged(tol) or
 * max_iter iterations, on a 1 x 1 cell with the default options otherwise;
 * its results are the one-site and the two nearest-neighbour RDMs.  Every
 * solve runs the same code on its own context as it would alone, so its
 * results do not depend on what else runs (bit for bit).
 *
 * The paper has no serving component: each solve is the CTMRG of Sec. II A
 * (in the eigenbasis of Sec. II B for CTM_FORM_Z2) run to the convergence
 * test of ctm_converged, and the calls below are the queueing, memory and
 * thread handling around such solves, defined by this library alone.
 *
 * All functions return CTM_OK or an error code of hctm.h.  One server may be
 * used from several host threads.
 */
#ifndef HCTM_SERVE_H
#define HCTM_SERVE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ctm_server ctm_server;

typedef struct {
  int status;        /* CTM_OK, or the error code that ended the solve */
  int iterations;    /* CTMRG iterations run */
  int converged;     /* 1 if delta < tol was reached */
  double delta;      /* delta after the last iteration (see ctm_converged) */
  double t_submit;   /* seconds since the server was created: submitted, */
  double t_start;    /* admitted (workspace taken), */
  double t_end;      /* results ready */
  char message[160]; /* error message if status != CTM_OK */
} ctm_solve_info;

/* Create a server on the current device with a device pool of pool_bytes
 * (allocated now) and at most max_active concurrent solves (1..64). */
int ctm_server_create(ctm_server** out, size_t pool_bytes, int max_active);

/* Queue a solve: A (host, d*D^4 doubles, legs [s,u,l,d,r], copied at the
 * call), form CTM_FORM_Z2 or CTM_FORM_DENSE, tol > 0, max_iter >= 1.  *id
 * identifies it for ctm_server_wait.  CTM_E_NOMEM if its workspace can never
 * fit into the pool; argument errors as for ctm_init. */
int ctm_server_submit(ctm_server* s, const double* A, int d, int D, int chi, int form, double tol, int max_iter,
                      long long* id);

/* Queue a solve of the complex tensor A_re + i A_im (host, d*D^4 doubles
 * each, copied; see ctm_init_complex: Z2 form, d <= 8); waited for like any
 * other solve, its imaginary RDM parts through ctm_server_wait_complex. */
int ctm_server_submit_complex(ctm_server* s, const double* A_re, const double* A_im, int d, int D, int chi,
                              double tol, int max_iter, long long* id);

/* Block until solve id has ended, then copy its results: rho1 (d*d), rho2_h
 * and rho2_v (d^4 each, the pairs (0,0)-(1,0) and (0,0)-(0,1)); any of them
 * may be NULL.  A solve can be waited for once; its results are released
 * afterwards.  Returns CTM_E_ARG for an unknown id, else CTM_OK (the solve's
 * own outcome is info->status). */
int ctm_server_wait(ctm_server* s, long long id, double* rho1, double* rho2_h, double* rho2_v,
                    ctm_solve_info* info);

/* The same with the imaginary parts (zero for a real tensor); any pointer may
 * be NULL. */
int ctm_server_wait_complex(ctm_server* s, long long id, double* rho1_re, double* rho1_im, double* rho2_h_re,
                            double* rho2_h_im, double* rho2_v_re, double* rho2_v_im, ctm_solve_info* info);

/* Number of solves waiting for admission and running now. */
int ctm_server_load(ctm_server* s, int* waiting, int* running);

/* Wait for every queued and running solve, then release everything; NULL is
 * accepted. */
void ctm_server_destroy(ctm_server* s);

#ifdef __cplusplus
}
#endif

#endif /* HCTM_SERVE_H */
