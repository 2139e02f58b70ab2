/* A C program on the C ABI alone (include/rc.h, librc.so, the HIP runtime): the ionospheric
 * correction of a single-bin tone, checked against its closed form.  For x[n] = exp(2 pi i k0 n / N)
 * the operator of Eq (16) returns H_k0 x[n] with H_k0 = exp(-i 4 pi K2 / (c f_k0)),
 * f_k0 = carrier + fs k0 / N (k0 < N / 2).  Prints "ok <max error>" and exits 0 when the largest
 * error is below 1e-5. */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "rc.h"

static const double kPi = 3.14159265358979323846;

int main(void)
{
    const int64_t n = 4096, k0 = 1234;
    const double fs = 10e6, fc = 450e6, tec = 50e16, c = 299792458.0;
    rc_c64 *x = (rc_c64 *)malloc(n * sizeof(rc_c64)), *y = (rc_c64 *)malloc(n * sizeof(rc_c64));
    for (int64_t i = 0; i < n; ++i) {
        const double a = 2.0 * kPi * (double)((k0 * i) % n) / (double)n;
        x[i].re = (float)cos(a);
        x[i].im = (float)sin(a);
    }
    rc_context ctx = NULL;
    if (rc_create(0, &ctx) != RC_OK) {
        fprintf(stderr, "rc_create failed\n");
        return 1;
    }
    void *dx = NULL, *dy = NULL;
    if (hipMalloc(&dx, n * sizeof(rc_c64)) != hipSuccess || hipMalloc(&dy, n * sizeof(rc_c64)) != hipSuccess) {
        fprintf(stderr, "hipMalloc failed\n");
        return 1;
    }
    if (hipMemcpy(dx, x, n * sizeof(rc_c64), hipMemcpyHostToDevice) != hipSuccess)
        return 1;
    rc_status st = correct_ionosphere(ctx, (const rc_c64 *)dx, (rc_c64 *)dy, n, fs, fc, tec, RC_CORRECT, NULL);
    if (st == RC_OK)
        st = rc_sync(ctx, NULL);
    if (st != RC_OK) {
        fprintf(stderr, "correct_ionosphere: %s: %s\n", rc_status_string(st), rc_last_error(ctx));
        return 1;
    }
    if (hipMemcpy(y, dy, n * sizeof(rc_c64), hipMemcpyDeviceToHost) != hipSuccess)
        return 1;
    const double f = fc + fs * (double)k0 / (double)n;
    const double ph = -4.0 * kPi * rc_k2_per_tec() * tec / (c * f);
    double err = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double a = 2.0 * kPi * (double)((k0 * i) % n) / (double)n + ph;
        const double dr = y[i].re - cos(a), di = y[i].im - sin(a);
        err = fmax(err, sqrt(dr * dr + di * di));
    }
    (void)hipFree(dx);
    (void)hipFree(dy);
    rc_destroy(ctx);
    free(x);
    free(y);
    printf("%s %.3e\n", err < 1e-5 ? "ok" : "FAIL", err);
    return err < 1e-5 ? 0 : 2;
}
