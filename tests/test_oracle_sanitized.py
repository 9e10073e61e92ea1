"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(a CPU build with gcc, no OpenMP): a driver calls every entry point of
oracle/lfo.h on small and degenerate grids (one cell, one row, one column),
every boundary pair, with and without mass fractions and with both
reconstructions, and the exact Riemann solver on a regular and a vacuum
case.  Any out-of-bounds access, leak, or undefined operation (signed
overflow, misaligned or null access, bad shift) aborts the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include "lfo.h"

static uint64_t s = 88172645463325252ull;
static double urand(double lo, double hi) {
    s ^= s << 13; s ^= s >> 7; s ^= s << 17;
    return lo + (hi - lo) * (double)(s >> 11) / 9007199254740992.0;
}

static int run(int nx, int ny, int bx, int by, int ns, int recon, double beta) {
    lfo_params P = {nx, ny, 1.0 / nx, 1.0 / (ny > nx ? ny : nx), 1.4, 0.5, beta, bx, by, ns, recon};
    const int nf = 4 + ns;
    const size_t N = (size_t)nx * ny, M = nf * N, M4 = 4 * N;
    double *U = malloc(sizeof(double) * M), *V = malloc(sizeof(double) * M), *R = malloc(sizeof(double) * M);
    double *a = malloc(sizeof(double) * M4), *b = malloc(sizeof(double) * M4), *c = malloc(sizeof(double) * M4);
    double *dts = malloc(sizeof(double) * 8), tot[4 + LFO_MAX_SPECIES];
    for (size_t q = 0; q < N; ++q) {
        double rho = urand(0.5, 1.5), u = urand(-1, 1), v = urand(-1, 1), p = urand(0.5, 1.5);
        U[q] = rho; U[N + q] = rho * u; U[2 * N + q] = rho * v;
        U[3 * N + q] = p / 0.4 + 0.5 * rho * (u * u + v * v);
        for (int k = 0; k < ns; ++k) U[(4 + k) * N + q] = rho * urand(0, 1);
    }
    double dt, t; int64_t n;
    if (lfo_residual(&P, U, R) || lfo_dt(&P, U, &dt) || lfo_step(&P, U, dt, V)) return 1;
    for (size_t q = 0; q < M; ++q) V[q] = U[q];
    if (lfo_advance(&P, V, 0.0, INFINITY, 3, &t, &n, dts) || n != 3) return 2;
    lfo_totals(&P, V, tot);
    if (ns == 0 && recon == LFO_RECON_PRIMITIVE) {
        for (size_t q = 0; q < M4; ++q) a[q] = urand(-1, 1);
        if (lfo_residual_jvp(&P, U, a, b) || lfo_residual_vjp(&P, U, a, c)) return 3;
        if (lfo_tlm_step(&P, U, dt, a, b) || lfo_adjoint_step(&P, U, dt, a, c)) return 4;
    } else if (lfo_residual_vjp(&P, U, U, c) != LFO_ERR_ARG) {
        return 5;
    }
    free(U); free(V); free(R); free(a); free(b); free(c); free(dts);
    return 0;
}

int main(void) {
    const int shapes[][2] = {{1, 1}, {1, 7}, {7, 1}, {5, 3}, {13, 11}};
    const double betas[] = {0.0, 1.0, 1.5, 2.0};
    for (int i = 0; i < 5; ++i)
        for (int bc = 0; bc < 4; ++bc)
            for (int v = 0; v < 3; ++v) {
                const int ns = v == 1 ? 2 : 0, recon = v == 2 ? LFO_RECON_CONSERVATIVE : LFO_RECON_PRIMITIVE;
                const int rc = run(shapes[i][0], shapes[i][1], bc & 1, bc >> 1, ns, recon, betas[(i + bc) % 4]);
                if (rc) { printf("failed %d at shape %d bc %d variant %d\n", rc, i, bc, v); return rc; }
            }
    double xi[5] = {-2, -0.5, 0, 0.5, 2}, r[5], u[5], p[5], ps, us;
    if (lfo_exact_riemann(1.4, 1, 0, 1, 0.125, 0, 0.1, 5, xi, r, u, p, &ps, &us)) return 6;
    if (lfo_exact_riemann(1.4, 1, -10, 0.4, 1, 10, 0.4, 5, xi, r, u, p, &ps, &us) != LFO_ERR_VACUUM) return 7;
    printf("ok\n");
    return 0;
}
"""


def _gcc_sanitizers(tmp):
    src = tmp / "probe.c"
    src.write_text("int main(void) { return 0; }\n")
    r = subprocess.run(["gcc", "-fsanitize=address,undefined", str(src), "-o", str(tmp / "probe")],
                       capture_output=True)
    return r.returncode == 0


def test_oracle_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None or not _gcc_sanitizers(tmp_path):
        pytest.skip("gcc with AddressSanitizer/UBSan is not available")
    drv = tmp_path / "drv.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "drv"
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-omit-frame-pointer",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", os.path.join(ROOT, "oracle"), os.path.join(ROOT, "oracle", "lfo.c"), str(drv),
                    "-lm", "-o", str(exe)], check=True, capture_output=True)
    # a library preloaded into every process need not come after the
    # sanitizer runtime: do not insist on the link order
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
