/*
 * vofserve: a continuous-batching request loop on top of libvofpoisson.
 *
 * Clients submit Poisson solves (the pressure solve of section 3.2) and
 * liquid-velocity extensions (section 3.6) of any supported grid, boundary
 * conditions and precision.  A scheduler thread owned by the server
 *   - keeps one or more plans (twiddles, eigenvalues, z coefficients,
 *     workspace) resident per request class (grid, dz, bc, precision) and
 *     admits work by the device bytes those plans hold: a new plan is created
 *     only while the resident plans fit in the configured budget, evicting idle
 *     plans least recently used first; requests wait while nothing can be
 *     evicted;
 *   - groups queued requests of one class and kind into batches of up to
 *     max_batch members, which run as one launch per pass
 *     (poisson_solve_batched / extend_liquid_velocity_batched);
 *   - runs batches on `lanes` HIP streams (at most two batches in flight per
 *     lane), so batches of different classes overlap on the device; requests
 *     that arrive while batches run join the next batch as soon as a lane and
 *     plan memory free up.
 * A member's result does not depend on the batch it ran in (the batched
 * kernels keep every member's arithmetic separate), so it equals the result of
 * the same request served alone, bit for bit.
 *
 * Field pointers in a request are DEVICE pointers owned by the client, which
 * keeps them valid and unmodified until the request's result has been
 * returned by vp_server_wait.  All calls are thread-safe.
 *
 * Timestamps are microseconds of vp_server_now_us (a monotonic host clock).
 */
#ifndef VOFSERVE_H
#define VOFSERVE_H

#include "vofpoisson.h"

#ifdef __cplusplus
extern "C" {
#endif

#define VP_EAGAIN (-5)    /* queue full (submit) or result not ready (wait) */
#define VP_ETOOBIG (-6)   /* the class's plan alone exceeds the memory budget */
#define VP_ECANCELED (-7) /* cancelled before it was dispatched */
#define VP_ETIMEDOUT (-8) /* not dispatched within its queue timeout */

#define VP_REQ_SOLVE 0  /* sol = L^+ rhs */
#define VP_REQ_EXTEND 1 /* extend_liquid_velocity with the fields in `ext` */

/* host-forced faults for failure-handling checks (vp_server_inject) */
#define VP_FAULT_LAUNCH 0 /* the next `count` batches fail at launch (VP_EHIP), no device work */
#define VP_FAULT_PLAN 1   /* the next `count` plan creations fail (VP_ENOMEM) */

typedef struct vp_server vp_server;

typedef struct vp_server_config {
  long long hbm_budget; /* device bytes the resident plans may hold (> 0) */
  int lanes;            /* HIP streams, 1..8 */
  int max_batch;        /* members per batch, 1..VP_MAX_BATCH */
  int max_pending;      /* queued (not yet dispatched) requests; beyond: VP_EAGAIN */
  int dry_run;          /* 1: no device calls at all; a batch takes dry_run_us */
  double dry_run_us;
} vp_server_config;

typedef struct vp_request {
  int kind;      /* VP_REQ_SOLVE or VP_REQ_EXTEND */
  int precision; /* VP_PRECISION_FP64 or VP_PRECISION_MIXED */
  int nx, ny, nz;
  double dx, dy;
  const double* dz;     /* HOST, nz cell widths (copied by submit) */
  const char* bc;       /* 3 or 6 letters as in poisson_plan_create (copied) */
  const double* rhs;    /* solve: device right-hand side */
  double* sol;          /* solve: device solution (may alias rhs) */
  vp_extend_fields ext; /* extend: device fields; phi required for mixed */
  double queue_timeout_ms; /* > 0: fail with VP_ETIMEDOUT if not dispatched in time */
} vp_request;

typedef struct vp_result {
  int status;         /* VP_OK, or the error the request ended with */
  int batch;          /* members of the batch it ran in (0 if never dispatched) */
  int lane;           /* lane it ran on (-1 if never dispatched) */
  double t_submit_us; /* accepted by vp_server_submit */
  double t_dispatch_us; /* its batch was launched (0 if never) */
  double t_done_us;   /* completion observed by the scheduler */
} vp_result;

typedef struct vp_server_stats {
  long long submitted, rejected, completed, failed, cancelled, timed_out;
  long long batches, batched_requests;
  long long plans_created, plans_evicted, plans_resident;
  long long bytes_resident, bytes_peak;
  long long pending, running; /* queued requests, batches in flight */
} vp_server_stats;

/* Monotonic host clock in microseconds (the clock of every timestamp). */
double vp_server_now_us(void);

/*
 * A new plan instance of a class whose plans are all busy is made only when
 * that class and kind have at least max_batch / 2 queued requests; a smaller
 * backlog waits for the busy plan's lane.
 *
 * Start a server on the current HIP device (none touched with dry_run).
 * Returns NULL and sets *status (VP_EINVAL for a bad configuration, VP_EHIP
 * if streams cannot be created).
 */
vp_server* vp_server_create(const vp_server_config* config, int* status);

/*
 * Queue one request; on VP_OK *ticket identifies it.  Rejected at once (and
 * counted as rejected) with VP_EINVAL (missing fields), VP_EUNSUPPORTED (grid
 * or bc, see poisson_plan_check), VP_ETOOBIG (plan footprint above the
 * budget) or VP_EAGAIN (max_pending requests already queued).
 */
int vp_server_submit(vp_server* server, const vp_request* request, long long* ticket);

/*
 * Create plans of the request's class (only its grid, dz, bc and precision
 * are read) until `instances` (1..lanes) exist, so that traffic of that class
 * finds them resident: a plan made while batches run stalls the scheduler
 * for the device allocation.  Waits up to timeout_ms (< 0: forever).
 * VP_OK (*created = plans made, may be NULL), VP_ETOOBIG if that many plans
 * exceed the budget, VP_EAGAIN on timeout, or the plan-creation status.
 */
int vp_server_prewarm(vp_server* server, const vp_request* request, int instances,
                      double timeout_ms, int* created);

/*
 * Wait up to timeout_ms (0: just look, < 0: forever) for a request to end.
 * VP_OK: *result is filled and the ticket is released (its fields may be
 * reused); VP_EAGAIN: still queued or running; VP_EINVAL: unknown ticket.
 */
int vp_server_wait(vp_server* server, long long ticket, double timeout_ms, vp_result* result);

/* Ask for a queued request to be dropped (it ends with VP_ECANCELED unless
 * it was dispatched first).  VP_EINVAL for an unknown ticket. */
int vp_server_cancel(vp_server* server, long long ticket);

/* Wait until nothing is queued or running (timeout_ms < 0: forever).
 * VP_OK, or VP_EAGAIN on timeout. */
int vp_server_drain(vp_server* server, double timeout_ms);

int vp_server_get_stats(vp_server* server, vp_server_stats* stats);

/* Force a fault from the host (VP_FAULT_*), for failure-handling checks. */
int vp_server_inject(vp_server* server, int fault, int count);

/* Drain, stop the scheduler and release every plan, stream and event. */
void vp_server_destroy(vp_server* server);

#ifdef __cplusplus
}
#endif

#endif /* VOFSERVE_H */
