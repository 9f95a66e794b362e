/*
 * abi_check.c -- the host-side argument checks of the C ABI (include/sidelobe.h)
 * under AddressSanitizer and UndefinedBehaviorSanitizer.  tests/test_sanitizers.py
 * links it against a host-sanitized build of the library; every call below must be
 * refused (or accepted, for the no-ops) before any device work, so it runs without
 * a GPU.
 */
#include <stdio.h>
#include <string.h>

#include "../../include/sidelobe.h"

static int fails = 0;
static void expect(int got, int want, const char *what) {
    if (got != want) {
        printf("%s: returned %d, expected %d (%s)\n", what, got, want, sc_last_error());
        ++fails;
    } else if (want != SC_OK && strlen(sc_last_error()) == 0) {
        printf("%s: no error message\n", what);
        ++fails;
    }
}

int main(void) {
    const int codes[] = {SC_OK, SC_EINVAL, SC_ENOMEM, SC_EHIP, SC_ESTATE, -99};
    for (unsigned i = 0; i < sizeof(codes) / sizeof(codes[0]); ++i)
        if (!sc_strerror(codes[i]) || !sc_strerror(codes[i])[0]) ++fails;
    sc_plan *p = 0;
    const int bad[][4] = {{-1, 0, 0, 0}, {10, -1, 0, 0}, {10, 11, 0, 0}, {10, 2, 7, 0}, {10, 2, 3, 0},
                          {10, 2, 0, 5}, {10, 2, 0, 18}, {8193, 2, 0, 0}, {500, 128, 1, 0}};
    for (unsigned i = 0; i < sizeof(bad) / sizeof(bad[0]); ++i)
        expect(sc_plan_create(&p, bad[i][0], bad[i][1], bad[i][2], bad[i][3], 0), SC_EINVAL, "sc_plan_create");
    expect(sc_plan_create(0, 4, 2, 0, 0, 0), SC_EINVAL, "sc_plan_create(NULL)");
    expect(sc_plan_destroy(0), SC_OK, "sc_plan_destroy(NULL)");
    expect(sc_set_sky_beam(0, 0, 0), SC_EINVAL, "sc_set_sky_beam(NULL)");
    expect(sc_interpolate(0, 0, 0, 0), SC_EINVAL, "sc_interpolate(NULL)");
    expect(sc_plan_build_psi_cube(0, 0), SC_EINVAL, "sc_plan_build_psi_cube(NULL)");
    expect(sc_interpolate_psi(0, 0, 0, 0), SC_EINVAL, "sc_interpolate_psi(NULL)");
    expect(sc_plan_info(0, 0, 0), SC_EINVAL, "sc_plan_info(NULL)");
    int64_t v = 0;
    expect(sc_plan_set_param(0, SC_PARAM_VALIDATE, 1), SC_EINVAL, "sc_plan_set_param(NULL)");
    expect(sc_plan_get_param(0, SC_PARAM_VALIDATE, &v), SC_EINVAL, "sc_plan_get_param(NULL)");
    expect(sc_plan_enable_timing(0, 1), SC_EINVAL, "sc_plan_enable_timing(NULL)");
    expect(sc_plan_convolve(0, 0, 0, 0, 0, 0), SC_EINVAL, "sc_plan_convolve(NULL)");
    expect(sc_convolve(0, 0, 4, 2, 0, -1, 0, 0, 0), SC_EINVAL, "sc_convolve(n < 0)");
    expect(sc_dipole_response(0, -1, 0, 0, 0, 0, 1, 1.0, 0.0, 0, 0), SC_EINVAL, "sc_dipole_response(lmax < 0)");
    expect(sc_dipole_response(0, 4, 2, 0, 0, 0, 0, 1.0, 0.0, 0, 0), SC_EINVAL, "sc_dipole_response(period 0)");
    sc_batch *b = 0;
    expect(sc_batch_create(&b, 0, 0, 100, SC_F64MAPS_F32GATHER, 0), SC_EINVAL, "sc_batch_create(ndet 0)");
    expect(sc_batch_create(0, 0, 1, 100, SC_F64MAPS_F32GATHER, 0), SC_EINVAL, "sc_batch_create(NULL)");
    expect(sc_batch_destroy(0), SC_OK, "sc_batch_destroy(NULL)");
    expect(sc_batch_run(0, 0, 0), SC_EINVAL, "sc_batch_run(NULL)");
    if (fails) return 1;
    printf("C ABI argument checks ran clean\n");
    return 0;
}
