/* Host-code check of plan creation under AddressSanitizer / UndefinedBehaviorSanitizer
 * (built by tests/test_host_sanitize.py, run on a machine without a GPU).
 *
 * The HIP calls that precede the first kernel launch are interposed: a "device" that
 * allocates from the host heap and fails the k-th allocation.  For every k, plan
 * creation must return NFFT_ERR_NOMEM, leave the output handle unset and free every
 * buffer it had allocated; past the last allocation the first launch fails (no device)
 * and the call returns NFFT_ERR_HIP, again with nothing left allocated.  Argument
 * errors and the no-device error of the real runtime are checked first.
 */
#include <stdio.h>
#include <stdlib.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>
#include "nfft.h"
/* interposed HIP calls: a device that allocates from the host heap and fails the n-th
   allocation */
static int n_alloc = 0, fail_at = 0, outstanding = 0;
hipError_t hipGetDevice(int *d) { *d = 0; return hipSuccess; }
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t a, int d) {
    (void)d;
    *v = a == hipDeviceAttributeMaxSharedMemoryPerBlock ? 163840 : 256;
    return hipSuccess;
}
hipError_t hipMalloc(void **p, size_t n) {
    if (++n_alloc == fail_at) { *p = 0; return hipErrorOutOfMemory; }
    *p = calloc(1, n ? n : 1);
    ++outstanding;
    return hipSuccess;
}
hipError_t hipFree(void *p) {
    if (p) { free(p); --outstanding; }
    return hipSuccess;
}
int main(void) {
    int64_t N[3] = {32, 32, 32};
    double fake[30] = {0};
    int fails = 0, nomem = 0;
    nfft_plan_t q = 0;
    if (nfft_plan_create(&q, 0, N, 10, fake, 4, 2.0, NFFT_C64, 0) != NFFT_ERR_ARG) ++fails;
    if (nfft_plan_create(&q, 2, N, 10, fake, 4, 1.0, NFFT_C64, 0) != NFFT_ERR_ARG) ++fails;
    if (nfft_plan_create(&q, 7, N, 10, fake, 4, 2.0, NFFT_C64, 0) != NFFT_ERR_UNSUPPORTED) ++fails;
    if (q) ++fails;
    for (int k = 1; k < 64; ++k) {
        nfft_plan_t p = 0;
        n_alloc = 0; fail_at = k; outstanding = 0;
        int rc = nfft_plan_create(&p, 3, N, 10, fake, 4, 2.0, NFFT_C128, 0);
        if (outstanding != 0 || p) { printf("k=%d rc=%d outstanding=%d\n", k, rc, outstanding); ++fails; }
        if (k <= n_alloc && rc == NFFT_ERR_NOMEM) ++nomem;
        else if (k <= n_alloc && rc != NFFT_ERR_NOMEM) { printf("k=%d rc=%d\n", k, rc); ++fails; }
        if (k > n_alloc) { printf("allocations before the first launch: %d; then rc=%d (%s)\n", n_alloc, rc, nfft_strerror(rc)); break; }
    }
    printf("injected failures returning NFFT_ERR_NOMEM: %d, fails %d\n", nomem, fails);
    if (nomem < 10) ++fails;
    return fails;
}
