/* gw_audit.h - launch audit of libgw, for tests and tooling.
 *
 * Not part of the method.  In audit mode every device buffer a context
 * allocates is host memory, copies are plain memcpy, and every kernel wrapper
 * stops after its host-side bounds guard: it computes the largest element
 * index the launch could touch in each buffer from the launch parameters and
 * refuses the launch when that index lies outside the buffer.  No kernel runs
 * and no result is computed, so every entry point that returns results
 * (gw_qp, gw_sigma, gw_wtable, gw_residues, gw_dielectric, gw_cholesky)
 * returns GW_EAUDIT once it has walked all of its launches; a refused launch
 * returns GW_EDEVICE with the guard's message in gw_last_error().  This walks
 * the whole host pipeline, for any problem size, on a machine without a GPU.
 * The same guards run before every real launch.
 */
#ifndef GW_AUDIT_H
#define GW_AUDIT_H

#ifdef __cplusplus
extern "C" {
#endif

#define GW_EAUDIT (-5)  /* audit mode: launches were checked, nothing was computed */

/* Switch the process into audit mode, irreversibly.  GW_EINVAL if any
 * context has been created in this process already. */
int gw_audit_enable(void);

/* Number of kernel launches checked (and skipped) in audit mode so far. */
long gw_audit_launch_count(void);

/* The server's grouped stage A on n caller-made contexts (gw_setup, closed
 * shell, the same padded shape and options, preconditioner on): builds a
 * temporary group for that shape and runs one batch of all n (as graphs
 * unless use_graph is 0), then frees the group.  rc[j]: 0 when context j's
 * W^c table (grid plus xi = 0) is now cached, or GW_ENOTSPD.  For tests and
 * the launch audit; returns GW_EINVAL for mismatched contexts. */
struct gw_ctx;
struct gw_grid;
int gw_group_stage_a(int n, struct gw_ctx* const* ctxs, const struct gw_grid* grid,
                     int use_graph, int* rc);

#ifdef __cplusplus
}
#endif
#endif /* GW_AUDIT_H */
