/* CPU oracle of the hotspot thermal stencil -- TEST INFRASTRUCTURE ONLY.
 *
 * The paper tunes a hotspot kernel from the BAT suite (Section 5; its tunable
 * parameters are Table 1) but does not define the computation, and the
 * suite's source is not available here. The computation is therefore the
 * compact thermal RC model of a chip (Huang et al., HotSpot, IEEE TVLSI 2006)
 * advanced by explicit (forward Euler) time steps, as the Rodinia suite uses
 * it: every cell of a rows x cols grid has a temperature T and a dissipated
 * power P, and one step sets
 *
 *   T'[r][c] = T + cc * ( P + (T[r-1][c] + T[r+1][c] - 2T) * gy
 *                           + (T[r][c-1] + T[r][c+1] - 2T) * gx
 *                           + (t_amb - T) * gz )
 *
 * with cc = dt / C (time step over the cell's heat capacity), gx and gy the
 * lateral thermal conductances between neighbouring cells along x (columns)
 * and y (rows), gz the vertical conductance to the ambient at t_amb. At the
 * chip edges a neighbour outside the grid is replaced by the cell itself (no
 * heat crosses the chip's sides). Every step reads only the previous step's
 * temperatures.
 *
 * Plain loops in FP64 (the inputs are FP32 values, widened), one step after
 * another, rows in parallel with OpenMP. It shares no code with the HIP path.
 */
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static long clampl(long v, long lo, long hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* One explicit step from cur to nxt (both rows x cols, FP64). */
static void hotspot_step_f64(const double *cur, const float *power, double *nxt, long rows, long cols, double cc,
                             double gx, double gy, double gz, double t_amb)
{
    long r;
#pragma omp parallel for schedule(static)
    for (r = 0; r < rows; ++r) {
        const long rn = clampl(r - 1, 0, rows - 1), rs = clampl(r + 1, 0, rows - 1);
        for (long c = 0; c < cols; ++c) {
            const long cw = clampl(c - 1, 0, cols - 1), ce = clampl(c + 1, 0, cols - 1);
            const double t = cur[r * cols + c];
            const double north = cur[rn * cols + c], south = cur[rs * cols + c];
            const double west = cur[r * cols + cw], east = cur[r * cols + ce];
            const double flow = (double)power[r * cols + c] + (north + south - 2.0 * t) * gy +
                                (west + east - 2.0 * t) * gx + (t_amb - t) * gz;
            nxt[r * cols + c] = t + cc * flow;
        }
    }
}

/* temp_out (FP64) = the grid after `steps` steps from temp_in. Returns 0, or
 * -1 for bad sizes, -2 when memory runs out. */
int oracle_hotspot_f64(const float *temp_in, const float *power, long rows, long cols, long steps, double cc,
                       double gx, double gy, double gz, double t_amb, double *temp_out)
{
    if (rows < 1 || cols < 1 || steps < 0) return -1;
    const size_t n = (size_t)rows * (size_t)cols;
    double *a = (double *)malloc(n * sizeof(double));
    double *b = (double *)malloc(n * sizeof(double));
    if (!a || !b) {
        free(a);
        free(b);
        return -2;
    }
    for (size_t k = 0; k < n; ++k) a[k] = (double)temp_in[k];
    for (long s = 0; s < steps; ++s) {
        hotspot_step_f64(a, power, b, rows, cols, cc, gx, gy, gz, t_amb);
        double *t = a;
        a = b;
        b = t;
    }
    memcpy(temp_out, a, n * sizeof(double));
    free(a);
    free(b);
    return 0;
}
