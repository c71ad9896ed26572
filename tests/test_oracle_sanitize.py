"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

Builds oracle/minimalist.c with gcc -fsanitize=address,undefined into a
small driver program and runs every entry point the tests use (both
drivers with level counters, intermediate movies and chains at every level,
the predicate probes) on degenerate and random inputs.  Any invalid access,
leak, signed overflow or shift error aborts the driver.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1205_1171_amd import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
int32_t oracle_sort(const int32_t*, int64_t, int32_t*);
int32_t oracle_hull(const int32_t*, int64_t, int32_t, int32_t*, int64_t, int64_t*, int64_t*, int32_t);
int32_t oracle_level_movies(const int32_t*, int64_t, int32_t, int32_t, int32_t*, int64_t, int64_t*, int64_t*);
int32_t oracle_level_chains(const int32_t*, int64_t, int32_t, int32_t, int32_t*, int32_t*);
int32_t oracle_predicate(const int64_t*, int32_t, int32_t);

static int levels(int64_t n) { int L = 0; while ((1LL << L) < n) ++L; return L; }

int main(int argc, char** argv) {
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t n;
    while (fread(&n, sizeof n, 1, f) == 1) {
        int32_t* p = malloc(sizeof(int32_t) * 3 * (n ? n : 1));
        if (fread(p, sizeof(int32_t), 3 * n, f) != (size_t)(3 * n)) return 3;
        int64_t cap = 2 * n > 0 ? 2 * n : 1, nf = 0;
        int L = levels(n) > 0 ? levels(n) : 1;
        int32_t* faces = malloc(sizeof(int32_t) * 3 * cap);
        int64_t* st = malloc(sizeof(int64_t) * 8 * L);
        int32_t* ord = malloc(sizeof(int32_t) * (n ? n : 1));
        if (oracle_sort(p, n, ord)) return 4;
        for (int flags = 0; flags < 8; ++flags) {
            if ((flags & 5) == 5) continue;
            if (oracle_hull(p, n, flags, faces, cap, &nf, (flags & 2) ? NULL : st, L)) return 5;
        }
        int32_t* ev = malloc(sizeof(int32_t) * 4 * cap);
        int64_t* bl = malloc(sizeof(int64_t) * (n ? n : 1));
        int32_t* pv = malloc(sizeof(int32_t) * (n ? n : 1));
        int32_t* nx = malloc(sizeof(int32_t) * (n ? n : 1));
        int64_t tot;
        for (int run = 0; run < 2; ++run)
            for (int k = -1; k <= levels(n); ++k) {
                if (oracle_level_movies(p, n, run, k, ev, cap, bl, &tot)) return 6;
                if (n > 0 && oracle_level_chains(p, n, run, k, pv, nx)) return 7;
            }
        for (int64_t t = 0; t + 6 <= n; t += 6) {
            int64_t rows[24];
            for (int q = 0; q < 6; ++q) {
                rows[4 * q] = p[3 * (t + q)]; rows[4 * q + 1] = p[3 * (t + q) + 1];
                rows[4 * q + 2] = p[3 * (t + q) + 2]; rows[4 * q + 3] = t + q;
            }
            for (int w = 0; w < 4; ++w) (void)oracle_predicate(rows, 6, w);
        }
        free(p); free(faces); free(st); free(ord); free(ev); free(bl); free(pv); free(nx);
    }
    fclose(f);
    puts("sanitized run ok");
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = tmp_path / "oracle_san"
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER)
    cmd = ["gcc", "-O1", "-g", "-std=gnu11", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-o", str(exe), str(drv),
           os.path.join(ROOT, "oracle", "minimalist.c")]
    try:
        subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    except subprocess.CalledProcessError as e:
        if b"asan" in e.stderr.lower() or b"sanitize" in e.stderr.lower():
            pytest.skip("gcc has no sanitizer runtime here")
        raise
    rng = np.random.default_rng(99)
    cases = [np.zeros((0, 3), np.int32), np.zeros((1, 3), np.int32), np.arange(6, dtype=np.int32).reshape(2, 3),
             np.array([[0, 0, 0], [5, 0, 1], [0, 7, 2]], np.int32), workloads.octahedron(3),
             workloads.cube_corners(5), workloads.moment_curve(-20, 20)]
    for t in range(24):
        n = int(rng.integers(3, 300))
        p = workloads.lattice(rng, n, [1, 2, 5, 40][t % 4])
        if t % 3 == 0:
            p[:, 0] = 7
        cases.append(p)
    cases.append(workloads.cube(rng, 500, 1 << 29))   # the coordinate bound
    cases.append(workloads.sphere(rng, 600, 1 << 20))
    data = tmp_path / "cases.bin"
    with open(data, "wb") as fh:
        for p in cases:
            p = np.ascontiguousarray(p, dtype="<i4")
            fh.write(np.int64(len(p)).tobytes())
            fh.write(p.tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe), str(data)], capture_output=True, timeout=600, env=env)
    assert r.returncode == 0, r.stderr.decode()[-4000:]
    assert b"sanitized run ok" in r.stdout
