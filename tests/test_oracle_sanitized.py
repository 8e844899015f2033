"""The oracle's C part built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, CPU only): every entry point runs on small grids, including lmax beyond
3 Nside - 1 and the polar rings of Nside 1024 where lambda_lm is carried in
scaled arithmetic, with no sanitizer report, and returns what the normal build
returns."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
SHT_C = os.path.join(os.path.dirname(HERE), "oracle", "sht.c")

# Reads the inputs the test wrote, calls each oracle entry point, writes the
# outputs one after another as doubles.
DRIVER = r"""
#include <stdio.h>
#include <stdlib.h>
void or_alm2map(int, int, const double*, double*, int);
void or_adjoint(int, int, const double*, double*, int);
void or_alm2map_rings(int, int, const double*, const int*, int, double*, int);
void or_adjoint_m(int, int, const double*, const int*, int, double*, int);
void or_lambda(int, double, double, int, double*);
void or_ring(int, int, double*, double*, long*, double*, long*);

static double* rd(FILE* f, long n) {
    double* p = (double*)malloc(sizeof(double) * (n > 0 ? n : 1));
    if (fread(p, sizeof(double), n, f) != (size_t)n) exit(3);
    return p;
}

int main(int argc, char** argv) {
    FILE* in = fopen(argv[1], "rb");
    FILE* out = fopen(argv[2], "wb");
    if (!in || !out) return 2;
    int hdr[2];
    while (fread(hdr, sizeof(int), 2, in) == 2) {
        int nside = hdr[0], lmax = hdr[1];
        long npix = 12L * nside * nside;
        long nalm = (long)(lmax + 1) * (lmax + 2) / 2;
        double* alm = rd(in, 2 * nalm);
        double* map = rd(in, npix);
        double* s = (double*)malloc(sizeof(double) * npix);
        double* b = (double*)malloc(sizeof(double) * 2 * nalm);
        or_alm2map(nside, lmax, alm, s, 2);
        or_adjoint(nside, lmax, map, b, 2);
        fwrite(s, sizeof(double), npix, out);
        fwrite(b, sizeof(double), 2 * nalm, out);
        int rings[2] = {4 * nside - 1, 1};
        double z, st, phi0; long n0, n1, start;
        or_ring(nside, rings[0], &z, &st, &n0, &phi0, &start);
        or_ring(nside, rings[1], &z, &st, &n1, &phi0, &start);
        double* sr = (double*)malloc(sizeof(double) * (n0 + n1));
        or_alm2map_rings(nside, lmax, alm, rings, 2, sr, 1);
        fwrite(sr, sizeof(double), n0 + n1, out);
        int ms[2] = {lmax, 0};
        long nb = (long)(lmax - ms[0] + 1) + (lmax - ms[1] + 1);
        double* bm = (double*)malloc(sizeof(double) * 2 * nb);
        or_adjoint_m(nside, lmax, map, ms, 2, bm, 1);
        fwrite(bm, sizeof(double), 2 * nb, out);
        free(alm); free(map); free(s); free(b); free(sr); free(bm);
    }
    /* polar rings of Nside 1024: values far below the double range on the way */
    double lam[2049];
    for (int r = 1; r <= 3; ++r) {
        double z, st, phi0; long n, start;
        or_ring(1024, r, &z, &st, &n, &phi0, &start);
        or_lambda(1000, z, st, 2048, lam);
        fwrite(lam, sizeof(double), 2049 - 1000, out);
    }
    fclose(in);
    fclose(out);
    return 0;
}
"""

CASES = [(1, 2), (2, 7), (4, 8), (8, 16)]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_c_under_address_and_undefined_sanitizers(tmp_path):
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "sanitized"
    subprocess.check_call(["gcc", "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-o", str(exe), str(drv), SHT_C, "-lm"])
    rng = np.random.default_rng(1702)
    inputs = []
    with open(tmp_path / "in.bin", "wb") as f:
        for nside, lmax in CASES:
            nalm = (lmax + 1) * (lmax + 2) // 2
            alm = rng.standard_normal((nalm, 2))
            alm[:lmax + 1, 1] = 0.0
            mp = rng.standard_normal(12 * nside * nside)
            np.array([nside, lmax], dtype=np.int32).tofile(f)
            alm.tofile(f)
            mp.tofile(f)
            inputs.append((nside, lmax, alm, mp))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    run = subprocess.run([str(exe), str(tmp_path / "in.bin"), str(tmp_path / "out.bin")],
                         env=env, capture_output=True, text=True, timeout=300)
    assert run.returncode == 0, run.stderr[-4000:]
    assert "runtime error" not in run.stderr and "ERROR: AddressSanitizer" not in run.stderr, \
        run.stderr[-4000:]

    got = np.fromfile(tmp_path / "out.bin", dtype=np.float64)
    pos = 0

    def take(n):
        nonlocal pos
        v = got[pos:pos + n]
        pos += n
        return v

    for nside, lmax, alm, mp in inputs:
        npix = 12 * nside * nside
        want_s = oracle.alm2map(alm, nside, lmax)
        want_b = oracle.adjoint(mp, nside, lmax)
        np.testing.assert_allclose(take(npix), want_s, rtol=0, atol=1e-13 * np.abs(want_s).max())
        np.testing.assert_allclose(take(want_b.size), want_b.ravel(), rtol=0,
                                   atol=1e-13 * np.abs(want_b).max())
        ring_vals = take(8)  # the last ring, then the first: 4 pixels each
        np.testing.assert_allclose(ring_vals[:4], want_s[-4:], rtol=0,
                                   atol=1e-13 * np.abs(want_s).max())
        np.testing.assert_allclose(ring_vals[4:], want_s[:4], rtol=0,
                                   atol=1e-13 * np.abs(want_s).max())
        bm = take(2 * (lmax + 2)).reshape(-1, 2)  # m = lmax (one l), then m = 0
        idx_mmax = oracle.alm_index(lmax, lmax, lmax)
        np.testing.assert_allclose(bm[0], want_b[idx_mmax], rtol=0, atol=1e-13 * np.abs(want_b).max())
        np.testing.assert_allclose(bm[1:], want_b[:lmax + 1], rtol=0, atol=1e-13 * np.abs(want_b).max())
    for r in (1, 2, 3):
        z, st = oracle.ring(1024, r)[:2]
        want = oracle.lambda_lm(1000, z, st, 2048)
        np.testing.assert_array_equal(take(2049 - 1000), want)
    assert pos == got.size
