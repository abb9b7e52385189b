/*
 * vofpoisson -- constant-coefficient Poisson solve, pressure projection and
 * liquid-velocity extension for MI355X (gfx950), C ABI.
 *
 * The operation (Scapin, Costa & Brandt, "A volume-of-fluid method for
 * interface-resolved simulations of phase-changing two-fluid flows"):
 *
 *  - section 3.2, pressure Poisson equation and velocity correction of the
 *    split projection: the variable-density pressure equation is split into a
 *    constant-coefficient Laplacian of p^{n+1} (solved directly) and an
 *    explicit term in the extrapolated pressure p_hat;
 *  - section 3.6, Stefan-flow potential, liquid-velocity extension and
 *    interface velocity: lap(phi) = s, u_1^e = u - grad(phi),
 *    u_Gamma = u_1^e - (mdot/rho1) n, with phi under the pressure's boundary
 *    conditions.
 *
 * Discretisation (section 3: fixed Cartesian grid, marker-and-cell layout,
 * second-order finite differences).  Fields are real, row-major with x
 * fastest: element (i, j, k) is at i + nx*(j + ny*k).  Cell-centred scalars
 * (p, p_hat, rho, s, phi) have nx*ny*nz entries; each face-velocity array
 * has nx*ny*nz entries too: u[i,j,k] is on face i+1/2, v on j+1/2, w on
 * k+1/2.  With a wall ('N') in a direction the face with the last index is
 * the wall; the face at -1/2 is implicit.  G is the face gradient (zero on
 * wall faces), D the cell divergence, L = D(G(.)).  An outflow end ('D', the
 * zero-pressure outflow boundary of the cases of section 4) puts p = 0 on the
 * boundary face, half a cell beyond the end centre: G there is
 * (0 - p_end) / (h/2) at an upper end and (p_end - 0) / (h/2) at a lower one,
 * and an upper outflow face's velocity is stored like any other face (the one
 * with the last index).  x and y are uniform
 * (dx, dy); z may be stretched: dz[k] is the width of cell k and the centre
 * distance across face k+1/2 is (dz[k] + dz[k+1]) / 2 (periodic z wraps).
 *
 * Without outflow ends the Poisson solve returns the unique p with
 *      L p = f - mean_W(f)   and   sum_k dV_k p_k = 0,
 * mean_W being the cell-volume-weighted mean.  A right-hand side with a
 * non-zero weighted mean is not an error: its mean is removed (and kept in
 * the plan as a diagnostic, poisson_plan_last_mean).  With an outflow end
 * anywhere L is non-singular and the solve returns p = L^-1 f (nothing is
 * removed; poisson_plan_last_mean gives 0).
 *
 * Pointers: every field pointer is a DEVICE pointer owned by the caller and
 * must stay valid until the work queued on `hip_stream` has completed.
 * `hip_stream` is a hipStream_t (NULL = the default stream).  All calls are
 * asynchronous (no host synchronisation).  A plan holds its own device
 * workspace, so one plan must not be used by two streams at the same time.
 *
 * Status codes: 0 ok; -1 invalid argument; -2 unsupported size or boundary
 * combination; -3 device out of memory; -4 HIP runtime error (the HIP
 * error string is kept per thread, see poisson_strerror).
 */
#ifndef VOFPOISSON_H
#define VOFPOISSON_H

#ifdef __cplusplus
extern "C" {
#endif

#define VP_OK 0
#define VP_EINVAL (-1)
#define VP_EUNSUPPORTED (-2)
#define VP_ENOMEM (-3)
#define VP_EHIP (-4)

#define VP_PRECISION_FP64 0
#define VP_PRECISION_MIXED 1

#define VP_MAX_BATCH 16 /* fields per batched call */

typedef struct poisson_plan poisson_plan;

/*
 * Create a plan on the current HIP device.
 *   nx, ny : a transform length: 2^k in [8, 1024], 3 * 2^k in [24, 768]
 *            or 5 * 2^k in [40, 640] (radix 2/4/8/16 passes after one
 *            radix-3 or radix-5 pass);
 *   nz     : >= 1 (>= 3 when z is periodic), at most 1024;
 *   dx, dy : > 0;  dz: HOST array of nz cell widths, each > 0 (copied);
 *   bc     : 3 characters for x, y, z (both ends alike) or 6 for the ends
 *            x-, x+, y-, y+, z-, z+ (either case): 'P' periodic (both ends
 *            of a direction), 'N' wall with zero normal gradient of p (zero
 *            normal velocity), 'D' outflow (p = 0 on the boundary face).
 *            Every direction takes P or any pair of N and D (a wall at one
 *            end and an outflow at the other: a quarter-wave cosine
 *            transform in x and y, the tridiagonal pass in z).
 *            The face at -1/2 of an outflow at a lower end has no slot in
 *            the face arrays: project, extend_liquid_velocity(_batched) and
 *            vof_step return VP_EUNSUPPORTED for such a plan, whose face
 *            stencils take the velocities of those faces as planes through
 *            project_lf, extend_liquid_velocity_lf and vof_step_lf; the
 *            solves accept every combination;
 *   precision : VP_PRECISION_FP64, or VP_PRECISION_MIXED (FP32 storage of
 *            the spectra between passes, FP64 arithmetic inside them,
 *            refined by FP64 defect-correction steps, see
 *            poisson_plan_set_mixed);
 *   max_batch : largest n accepted by the batched calls, 1..VP_MAX_BATCH.
 * Allocates the plan's device tables and workspace: one spectrum slot of
 * 8*nx*ny*nz bytes per batch member for FP64, plus an FP32 spectrum slot per
 * member for mixed (poisson_plan_footprint gives the exact total).
 * Returns NULL and sets *status on failure (status may be NULL):
 * VP_EINVAL for bad arguments, VP_EUNSUPPORTED for sizes or boundary
 * conditions outside the limits above.
 */
poisson_plan* poisson_plan_create(int nx, int ny, int nz, double dx, double dy,
                                  const double* dz, const char* bc, int precision,
                                  int max_batch, int* status);

/*
 * Check the arguments of poisson_plan_create without touching the device:
 * VP_OK, VP_EINVAL or VP_EUNSUPPORTED, exactly as poisson_plan_create would
 * return them.
 */
int poisson_plan_check(int nx, int ny, int nz, double dx, double dy, const double* dz,
                       const char* bc, int precision, int max_batch);

/* Release every device allocation of the plan (synchronises the device). */
void poisson_plan_destroy(poisson_plan* plan);

/*
 * Poisson solve (the direct constant-coefficient solver of section 3.2):
 * sol = L^+ rhs as defined above.  rhs and sol: device, nx*ny*nz doubles;
 * sol may alias rhs.
 */
int poisson_solve(poisson_plan* plan, const double* rhs, double* sol, void* hip_stream);

/*
 * n independent solves with the plan's shape (0 <= n <= max_batch) in one
 * launch per pass: rhs and sol are HOST arrays of n device pointers.  Each
 * result equals that of poisson_solve on the same input, bit for bit (no
 * arithmetic depends on the other members).  sol[i] may alias rhs[i].
 */
int poisson_solve_batched(poisson_plan* plan, int n, const double* const* rhs,
                          double* const* sol, void* hip_stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the FP64
 * solve of poisson_solve, the same kernels and the same result bit for bit,
 * with its spectrum in a static device array of the library instead of the
 * plan's workspace.  The call allocates nothing and leaves the plan's
 * workspace untouched.  The array holds VP_NOALLOC_MAX_POINTS doubles
 * (64 MiB); every GPU the library runs on holds its own copy until the
 * process ends (its address is taken once per device when the first plan is
 * created there).  All calls on one GPU share that array, which keeps the
 * last call's contents: calls that overlap on one GPU (two streams, or two
 * host threads) race and must be serialised by the caller.
 *   plan : an FP64 plan on the current device with nx*ny*nz at most
 *          VP_NOALLOC_MAX_POINTS (VP_EUNSUPPORTED otherwise: a mixed plan or
 *          a larger grid; VP_EINVAL if another device is current);
 *   rhs, sol, hip_stream : as for poisson_solve (sol may alias rhs).
 */
#define VP_NOALLOC_MAX_POINTS 8388608 /* 2^23 points, e.g. 256 x 256 x 128 */
int poisson_solve_noalloc(poisson_plan* plan, const double* rhs, double* sol, void* hip_stream);

/*
 * Pressure projection of section 3.2 (constant-coefficient split):
 *   b   = rho0 D[(1/rho0 - 1/rho_f) G p_hat] + (rho0/dt) (D u* - s)
 *   p   = Poisson solve of b
 *   u  <- u* - dt [ (1/rho0) G p + (1/rho_f - 1/rho0) G p_hat ]
 * rho_f is the mean of the two cell densities sharing a face.
 *   u, v, w : in u*, out u^{n+1} (device, overwritten in place);
 *   phat, rho : device cell fields; rho0 > 0 (the smaller phase density);
 *   src : device s = mdot (1/rho2 - 1/rho1) |grad C|, or NULL for s = 0;
 *   dt > 0;  p : device output pressure (must not alias the inputs).
 */
int project(poisson_plan* plan, double* u, double* v, double* w,
            const double* phat, const double* rho, double rho0,
            const double* src, double dt, double* p, void* hip_stream);

/*
 * Velocities on the faces at -1/2 of the outflow ends at a lower end (the
 * zero-pressure outflow boundaries of section 4 on every side of a box): the
 * face arrays hold the faces i+1/2 .. n-1/2 only, so each such face set is a
 * DEVICE plane of its own, caller-owned:
 *   u : x = -1/2, ny*nz values, face (j, k) at j + ny*k;
 *   v : y = -1/2, nx*nz values, face (i, k) at i + nx*k;
 *   w : z = -1/2, nx*ny values, face (i, j) at i + nx*j.
 * An input set holds a plane exactly for the directions whose lower end is an
 * outflow (NULL for the others; VP_EINVAL otherwise); an output set may leave
 * such a plane NULL (not written).  On those faces p, p_hat and phi are 0
 * (G q = (q_first - 0) / (h/2), h the first cell's width) and rho is the first
 * cell's, as at an upper outflow face.
 */
typedef struct vp_lower_faces {
  double *u, *v, *w;
} vp_lower_faces;

/*
 * project with the lower outflow faces' velocities: `lower` (in u*, out
 * u^{n+1}, in place) as described above; otherwise as project.
 */
int project_lf(poisson_plan* plan, double* u, double* v, double* w,
               const vp_lower_faces* lower, const double* phat, const double* rho,
               double rho0, const double* src, double dt, double* p, void* hip_stream);

/*
 * Liquid-velocity extension of section 3.6:
 *   phi = Poisson solve of src;  u_1^e = u - G phi;  u_Gamma = u_1^e - q.
 *   u, v, w   : device input velocity (one-fluid, after projection);
 *   src       : device s = mdot (1/rho2 - 1/rho1) |grad C| (cell centres);
 *   qx,qy,qz  : device (mdot/rho1) n on faces, or all NULL (then ug, vg, wg
 *               must be NULL too);
 *   ue,ve,we  : device outputs u_1^e (may alias u, v, w);
 *   ug,vg,wg  : device outputs u_Gamma, or NULL;
 *   phi       : device output potential, or NULL (then the plan workspace
 *               holds it until the next call).
 */
int extend_liquid_velocity(poisson_plan* plan, const double* u, const double* v,
                           const double* w, const double* src,
                           const double* qx, const double* qy, const double* qz,
                           double* ue, double* ve, double* we,
                           double* ug, double* vg, double* wg,
                           double* phi, void* hip_stream);

/*
 * extend_liquid_velocity with the lower outflow faces: `lower` (in, u on
 * those faces) and `lower_e` (out, u_1^e there, which is also u_Gamma: q is 0
 * on a non-periodic boundary face; may alias `lower`); otherwise as
 * extend_liquid_velocity.
 */
int extend_liquid_velocity_lf(poisson_plan* plan, const double* u, const double* v,
                              const double* w, const vp_lower_faces* lower,
                              const double* src, const double* qx, const double* qy,
                              const double* qz, double* ue, double* ve, double* we,
                              const vp_lower_faces* lower_e, double* ug, double* vg,
                              double* wg, double* phi, void* hip_stream);

/* The device fields of one extension (same meaning as the arguments above). */
typedef struct vp_extend_fields {
  const double *u, *v, *w, *src, *qx, *qy, *qz;
  double *ue, *ve, *we, *ug, *vg, *wg, *phi;
} vp_extend_fields;

/*
 * n extensions with the plan's shape (0 <= n <= max_batch): the n Poisson
 * solves share one launch per pass, then the extension stencil runs per
 * member.  fields: HOST array of n structs.  With phi NULL (FP64 plans only)
 * member i's potential stays in workspace slot i.  Results equal those of
 * extend_liquid_velocity member by member, bit for bit.
 */
int extend_liquid_velocity_batched(poisson_plan* plan, int n, const vp_extend_fields* fields,
                                   void* hip_stream);

/*
 * One time step of the path: the projection of section 3.2 followed by the
 * extension of section 3.6 applied to the projected velocity.  Equivalent to
 * project(plan, u, v, w, phat, rho, rho0, src_p, dt, p) followed by
 * extend_liquid_velocity(plan, u, v, w, src_ext, q, ue, ug, phi), with the
 * correction and extension stencils fused into one pass over the faces.
 *   u, v, w    : in u*, out u^{n+1} (device, in place);
 *   src_p      : source of the pressure equation, or NULL (s = 0);
 *   src_ext    : source of the Stefan potential (required; in the paper the
 *                same field mdot (1/rho2 - 1/rho1) |grad C| as src_p);
 *   p, phi     : device outputs (distinct buffers);
 *   ue,ve,we   : device outputs u_1^e, or all NULL;
 *   qx..wg     : as in extend_liquid_velocity.
 */
int vof_step(poisson_plan* plan, double* u, double* v, double* w, const double* phat,
             const double* rho, double rho0, const double* src_p, double dt, double* p,
             const double* src_ext, const double* qx, const double* qy, const double* qz,
             double* ue, double* ve, double* we, double* ug, double* vg, double* wg,
             double* phi, void* hip_stream);

/*
 * vof_step with the lower outflow faces: `lower` (in u*, out u^{n+1}, in
 * place) and `lower_e` (out u_1^e = u_Gamma on those faces, may be NULL);
 * otherwise as vof_step.
 */
int vof_step_lf(poisson_plan* plan, double* u, double* v, double* w,
                const vp_lower_faces* lower, const double* phat, const double* rho,
                double rho0, const double* src_p, double dt, double* p,
                const double* src_ext, const double* qx, const double* qy,
                const double* qz, double* ue, double* ve, double* we,
                const vp_lower_faces* lower_e, double* ug, double* vg, double* wg,
                double* phi, void* hip_stream);

/*
 * Interface terms from the volume fraction (section 3.2: the regularised
 * delta |grad C| by Youngs' finite differences; section 3.4: the normal from
 * the gradient of C; section 3.6: the Stefan source and the jump of the
 * interface velocity), one pass over the fields.  The normal is
 * n = -grad C / |grad C|: it points into phase 2, as the jump condition of
 * section 2 (eq. rankine) orients it, since C is 1 in phase 1; so for mdot > 0
 * (evaporation) u_Gamma = u_1^e - q moves the interface into the liquid:
 *   s  = mdot (1/rho2 - 1/rho1) |grad C|            (cell centres),
 *   q  = (mdot / rho_e) n on the faces (qx on i+1/2, qy on j+1/2, qz on k+1/2):
 *        the mean of the two adjacent cells' values, 0 on a non-periodic
 *        boundary face (n = 0 where grad C = 0).
 * grad C at a cell centre is the mean of the gradients at its eight corners,
 * each taken from the eight cells around the corner (dx, dy and the z centre
 * distances), with periodic copies or mirrored values (zero normal gradient)
 * beyond the domain; on a uniform grid that is the central difference
 * weighted (1, 2, 1) in each transverse direction.  s and q are the src and
 * q arguments of project / extend_liquid_velocity / vof_step.
 *   C, mdot : device cell fields (volume fraction of phase 1, mass flux);
 *   rho1, rho2 > 0 : the two densities;
 *   phase : the phase whose divergence-free velocity extension builds the
 *           interface velocity: 1 (the liquid, section 3.6; rho_e = rho1) or
 *           2 (the vapour, for boiling, appendix A; rho_e = rho2).  The
 *           potential and the extension u - grad phi are the same for both;
 *           only the jump q changes;
 *   s, qx, qy, qz : device outputs (must not alias C or mdot).
 */
int interface_terms(poisson_plan* plan, const double* C, const double* mdot, double rho1,
                    double rho2, int phase, double* s, double* qx, double* qy, double* qz,
                    void* hip_stream);

/*
 * vof_step with the interface terms formed inside the step's first and last
 * passes (sections 3.2 and 3.6; the same terms as interface_terms): the
 * right-hand-side pass takes |grad C| by Youngs' differences and writes
 * s = mdot (1/rho2 - 1/rho1) |grad C| to `s` (the source of the pressure
 * equation and the right-hand side of the Stefan potential), then the two
 * solves run, then the epilogue forms q = (mdot / rho_e) n on the faces from
 * C and mdot and writes u_Gamma = u_1^e - q.  The fields s and q never make
 * a separate pass.  Same bits as interface_terms followed by vof_step with
 * src_p = src_ext = s and that q.
 *   u, v, w : u* in, u^{n+1} out (in place); phat, rho, rho0, dt as vof_step;
 *   C, mdot, rho1, rho2, phase : as interface_terms;
 *   p, phi, s : device outputs (distinct); ue, ve, we : optional (all or none);
 *   ug, vg, wg : required.
 * VP_EUNSUPPORTED for a plan with an outflow at a lower end (use
 * interface_terms and vof_step_lf), VP_EINVAL for bad arguments.
 */
int vof_step_interface(poisson_plan* plan, double* u, double* v, double* w, const double* phat,
                       const double* rho, double rho0, const double* C, const double* mdot,
                       double rho1, double rho2, int phase, double dt, double* p, double* s,
                       double* ue, double* ve, double* we, double* ug, double* vg, double* wg,
                       double* phi, void* hip_stream);

/*
 * VoF advection of section 3.1: C^{n+1} from C^n and the interface velocity
 * u_Gamma of section 3.6 (eq. cadv) by directional splitting, x then y then
 * z, each sweep implicit in its own result through the divergence of its
 * velocity component (eq. fluxes), then the final correction
 *   deflation = 1: C^{n+1} = C*** - dt F + dt C^{n+1} div(u_Gamma)  (eq. final_corr_2),
 *   deflation = 0: C^{n+1} = C*** - dt F                            (eq. final_corr_1),
 * F = C* du/dx + C** dv/dy + C*** dw/dz.  The fluxes are those of the MTHINC
 * method the paper cites (Ii et al. 2012), linear reconstruction: in a cell
 * of local coordinates X in [-1/2, 1/2]^3, H = 1/2 (1 + tanh(beta (m.X + d))),
 * m the unit Youngs normal in cell coordinates (dx g_x, dy g_y, dz_k g_z),
 * d fixed by the cell's volume; integrals of H exact along the dominant
 * axis of m and 2-point Gauss-Legendre in the other two; a face's flux is
 * sign(V) h times the integral of H over the part of the upwind cell the
 * face sweeps in dt.  Cells with C within 1e-8 of 0 or 1 (or a change of C
 * across the cell below 1e-12) are uniform; ghost cells beyond a
 * non-periodic end are uniform with the end cell's C.
 *   C      : device volume fraction C^n (cell centres);
 *   ug,vg,wg : device interface velocity on the faces (u_Gamma of
 *            extend_liquid_velocity / vof_step), zero on wall faces;
 *   lower  : u_Gamma on the faces at -1/2 of lower outflow ends (an input
 *            set, see vp_lower_faces), NULL for a plan without them;
 *   dt > 0 : time step, with |V| dt at most the upwind cell's width along
 *            each sweep (one cell per step; larger steps are clamped to it);
 *   beta > 0 : sharpness of the tanh profile (1 is the usual choice);
 *   deflation : 1 (the paper's method) or 0;
 *   C_new  : device output C^{n+1} (must not alias C).
 * Uses workspace slot 0 of the plan (C** between the sweeps).  VP_EUNSUPPORTED
 * for a plan with an outflow at a lower end and lower == NULL.
 */
int vof_advect(poisson_plan* plan, const double* C, const double* ug, const double* vg,
               const double* wg, const vp_lower_faces* lower, double dt, double beta,
               int deflation, double* C_new, void* hip_stream);

/*
 * Mixed-precision control (plans created with VP_PRECISION_MIXED).  A mixed
 * solve is p_0 = S32(f) followed by at most dc_steps FP64 defect-correction
 * steps p_k = p_{k-1} + e_k, e_k = S32(f - L_h p_{k-1}), where S32 is the
 * solve with FP32 spectra stored between its passes (FP64 arithmetic and
 * tables inside each pass) and the defect is formed in FP64 inside the first
 * pass of the correction.  After each correction the relative error left by
 * its FP32 solve is estimated as 2^-23 (G |f - L_h p_{k-1}| + |e_k|) / |p_k|,
 * G a constant of the plan (the largest RMS of 1/|lambda| over the z modes
 * of one (kx, ky) line: the FP32 rounding of the forward passes is
 * independent along z within a line); a member stops, on the device and
 * without a host synchronisation, once that is at most the tolerance.
 *   poisson_plan_set_mixed     : the most steps, 0..8 (default 3);
 *   poisson_plan_set_mixed_tol : the tolerance (default 1e-11); <= 0 runs
 *                                every step;
 *   poisson_plan_mixed_report  : steps taken and the last estimate of each of
 *                                the n members of the last mixed call
 *                                (host arrays, may be NULL; synchronises
 *                                hip_stream).
 * Each returns VP_EINVAL for an FP64 plan or a bad argument.
 */
int poisson_plan_set_mixed(poisson_plan* plan, int dc_steps);
int poisson_plan_set_mixed_tol(poisson_plan* plan, double tol);
int poisson_plan_mixed_report(poisson_plan* plan, int n, int* steps, double* estimate,
                              void* hip_stream);

/*
 * Weighted mean removed from the last right-hand side solved with this plan
 * (copied from the device: synchronises `hip_stream`).  Returns a status.
 */
int poisson_plan_last_mean(poisson_plan* plan, double* mean_out, void* hip_stream);

/*
 * Size in bytes of the device memory a plan with these arguments holds
 * (-1 for invalid arguments); poisson_plan_device_bytes gives it for an
 * existing plan.
 */
long long poisson_plan_footprint(int nx, int ny, int nz, int precision, int max_batch);
long long poisson_plan_device_bytes(const poisson_plan* plan);

/*
 * Launch-shape tuning (results do not change beyond rounding order, only speed):
 *   "x_radix", "y_radix" : values per thread of the radix schedule of the x
 *                 and y transform passes, 16 (radix-16 passes, default) or 8
 *                 (radix-8 passes: fewer registers and LDS per line, more
 *                 blocks per compute unit);
 *   "z_lines"   : lines per block of the tridiagonal z pass, 8, 16 (default)
 *                 or 32 (capped so that lines * segments <= 512);
 *   "z_spectral": 1 (default where possible) solves a uniform z grid with nz a
 *                 transform length (as nx, ny) and the same condition at both
 *                 ends by a real DFT (periodic), DCT-II (walls) or DST-II
 *                 (outflow) along z, a division by the 3-D eigenvalue and the
 *                 inverse transform, in one pass; 0 uses the tridiagonal pass
 *                 (VP_EUNSUPPORTED for 1 on other grids);
 *   "z_radix"   : values per thread of the spectral z pass, 16 or 8;
 *   "y_lines", "z_spectral_lines" : column pairs per block of the y passes
 *                 and of the spectral z pass (a power of two up to 256; 0, the
 *                 default: 256 threads' worth at radix 16; narrower tiles use
 *                 less LDS, so more blocks fit on a compute unit);
 *   "stencil_planes" : z-planes marched by one block of the right-hand-side
 *                 kernel (1..nz; default chosen for ~16k blocks);
 *   "stream_planes", "stream_tiled" : the correction and extension kernels
 *                 of project / extend_liquid_velocity: z-planes marched by one
 *                 block (1..nz, default 1) and LDS-staged 64 x 8 (or 16) tiles
 *                 where they fit (default 8; 0: plain one-row tiles; same bits);
 *   "epilogue_tiled", "epilogue_planes" : the fused epilogue of vof_step on
 *                 LDS-staged 64 x 8 (or 16) tiles marching that many planes
 *                 (defaults 8 and 1; tiled 0: plain one-row tiles; results
 *                 are bit-identical);
 *   "z_segment" : rows per segment of the partitioned tridiagonal z solve,
 *                 8 or 16 (at most 64 segments; default 8 on stretched grids
 *                 with nz <= 512, else 16; the autotuner tries both);
 *   "interface_planes" : z-planes marched by one block of interface_terms
 *                 (1..nz; default 64, halved down to 8 while the grid would
 *                 give fewer than 512 blocks, at most nz; results are
 *                 bit-identical);
 *   "interface_tile" : tile width of interface_terms (8, 16, 32 or 64, at
 *                 most the largest power of two dividing nx, the default;
 *                 the tile holds 512 cells; results are bit-identical);
 *   "rhs_tiled" : 8 (default) or 16 assembles the projection's right-hand
 *                 side on LDS-staged 64 x 8 (x 16) tiles where nx % 64 == 0 and
 *                 ny divides by the tile height (bit-identical results), 0 on
 *                 plain 64 x 4 tiles.
 * Returns VP_EINVAL for an unknown key or value.
 */
int poisson_plan_tune(poisson_plan* plan, const char* key, int value);

/* Current value of a tuning key (see poisson_plan_tune). */
int poisson_plan_get_tuning(poisson_plan* plan, const char* key, int* value);

/*
 * Autotuner: times every candidate of each knob above on the plan's own
 * workspace (which it overwrites) for a batch of nb fields, on hip_stream
 * (synchronising it), median of 5 runs each, one knob after another (x
 * radix, y radix, z lines, stencil planes; the last only when the
 * workspace holds a second field: mixed plans or max_batch >= 2), then,
 * where the spectral z pass applies, the fastest of the tuned tridiagonal
 * pass and the spectral pass at either radix and three tile widths (the y
 * tile width is tuned after the y radix); it leaves each at its fastest
 * value.  chosen (may be NULL) receives eight values: x_radix, y_radix,
 * z_lines, stencil_planes, z_spectral, z_radix, y_lines, z_spectral_lines.
 * Not for use while other calls on the plan run.
 */
int poisson_plan_autotune(poisson_plan* plan, int nb, void* hip_stream, int* chosen);

/*
 * Per-launch timing.  class_mask selects kernel classes (bit c for class c;
 * -1 for all, 0 to stop): every launch of a selected class is bracketed by
 * two HIP events recorded on the caller's stream (a small launch overhead).  poisson_plan_kernel_times waits for the recorded events,
 * writes per kernel class the total milliseconds and the launch count into
 * total_ms[0..n) and launches[0..n) (classes beyond n are dropped), and
 * forgets the recorded launches.  Classes are numbered 0..VP_NUM_KERNEL_CLASSES-1;
 * poisson_kernel_class_name gives their names (NULL outside that range).
 */
#define VP_NUM_KERNEL_CLASSES 19
int poisson_plan_set_profiling(poisson_plan* plan, int class_mask);
int poisson_plan_kernel_times(poisson_plan* plan, double* total_ms, int* launches, int n);
const char* poisson_kernel_class_name(int cls);

/* Human-readable text for a status code (for VP_EHIP: the last HIP error). */
const char* poisson_strerror(int status);

/* Library version string. */
const char* vofpoisson_version(void);

#ifdef __cplusplus
}
#endif

#endif /* VOFPOISSON_H */
