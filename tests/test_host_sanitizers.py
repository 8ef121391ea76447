"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the oracle's solver paths (every dimension, boundary condition and
WENO order, whole domain and sub-box) and the library's host sampler are
built with gcc/g++ and the sanitizers, run on small cases, and must finish
without a report (out-of-bounds access, use after free, leak, signed
overflow, misaligned or null access)."""
import os
import shutil
import subprocess
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]

ORACLE_DRIVER = r"""
#include "ORACLE_C"
#include <stdio.h>

static void run(int nd, int n, int bc, int order)
{
    orc_spec s;
    memset(&s, 0, sizeof s);
    s.ndim = nd; s.n = n; s.bc = bc; s.n_sub = 2; s.cfl = 0.3;
    s.gamma1 = 6.12; s.pc1 = 3.43e8; s.gamma2 = 1.4; s.pc2 = 0.0;
    s.rho1 = 1000.0; s.rho2 = 1.0; s.p_bubble = 2340.0; s.p_inf = 1.0e7;
    s.center[0] = s.center[1] = s.center[2] = 0.5;
    s.cloud_radius = 0.3; s.ramp_delta = 0.015; s.ramp_width = 0.1;
    s.weno_eps = 1e-6; s.weno_order = order;
    double bub[2][4] = { { 0.45, 0.5, 0.5, 0.08 }, { 0.62, 0.55, 0.5, 0.05 } };
    if (nd < 3) { bub[0][2] = 0.0; bub[1][2] = 0.0; }
    int64_t nc = 1;
    for (int a = 0; a < nd; ++a) nc *= n;
    int nv = 4 + nd;
    double* U = (double*)malloc(sizeof(double) * nv * nc);
    orc_box box;
    for (int a = 0; a < 3; ++a) { box.lo[a] = 0; box.len[a] = a < nd ? n : 1; }
    orc_init(&s, &box, &bub[0][0], 2, U);
    orc_qoi q;
    orc_solve(&s, U, 0.0, 3, 100, &q);
    orc_reduction r;
    orc_initial_reduction(&s, &bub[0][0], 2, &r);
    double dts[2];
    orc_run_steps(&s, U, 2, dts);
    if (bc != 1) {
        /* a sub-box away from the low corner, with the same step sizes */
        orc_box sb;
        for (int a = 0; a < 3; ++a) { sb.lo[a] = a < nd ? 2 : 0; sb.len[a] = a < nd ? n - 3 : 1; }
        int64_t sc = 1;
        for (int a = 0; a < nd; ++a) sc *= n - 3;
        double* V = (double*)malloc(sizeof(double) * nv * sc);
        orc_box_steps(&s, &sb, &bub[0][0], 2, 2, dts, V);
        free(V);
    }
    free(U);
    printf("ok %d %d %d %d status %d\n", nd, n, bc, order, q.status);
}

int main(void)
{
    for (int bc = 0; bc < 3; ++bc)
        for (int order = 3; order <= 5; order += 2) {
            run(1, 24, bc, order);
            run(2, 12, bc, order);
            run(3, 8, bc, order);
        }
    return 0;
}
"""

SAMPLER_DRIVER = r"""
#include <cstdarg>
#include <cstdio>
#include <vector>
#include "ofm.h"
#include "ofm_error.h"

namespace ofm {
int fail(ofm_ctx*, int code, const char*, ...) { return code; }
}

int main()
{
    ofm_cloud_spec c = {};
    int bad = 0;
    for (int nd = 1; nd <= 3; ++nd)
        for (int nb : {0, 1, 8, 50}) {
            c.ndim = nd; c.n_bubbles = nb; c.cloud_radius = 0.3;
            c.center[0] = c.center[1] = c.center[2] = 0.5;
            c.r_median = 0.015; c.r_sigma = 0.1; c.r_lo = 0.012; c.r_hi = 0.018;
            std::vector<double> out(4 * (nb + 1), -1.0);
            // 50 non-overlapping bubbles do not fit on a 1-D segment of 0.6:
            // the sampler gives up with OFM_EINFEASIBLE
            const int want = (nd == 1 && nb == 50) ? OFM_EINFEASIBLE : 0;
            for (unsigned i = 0; i < 3; ++i)
                if (ofm_sample_cloud(&c, 170504374ull, 1, i, out.data()) != want) ++bad;
        }
    c.ndim = 4;                                   // rejected, not read past
    std::vector<double> out(8);
    if (ofm_sample_cloud(&c, 1, 0, 0, out.data()) == 0) ++bad;
    if (ofm_sample_cloud(nullptr, 1, 0, 0, out.data()) == 0) ++bad;
    std::printf("sampler bad=%d\n", bad);
    return bad;
}
"""


def _have(tool, lang, tmp_path):
    if shutil.which(tool) is None:
        return False
    src = tmp_path / ("probe." + lang)
    src.write_text("int main(void){return 0;}\n")
    r = subprocess.run([tool] + SAN + [str(src), "-o", str(tmp_path / "probe")], capture_output=True)
    return r.returncode == 0


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    return r


def test_oracle_under_sanitizers(tmp_path):
    if not _have("gcc", "c", tmp_path):
        pytest.skip("gcc with ASan/UBSan not available")
    drv = tmp_path / "oracle_driver.c"
    drv.write_text(ORACLE_DRIVER.replace("ORACLE_C", os.path.join(ROOT, "oracle", "flow_oracle.c")))
    exe = tmp_path / "oracle_driver"
    subprocess.run(["gcc", "-std=c99", "-ffp-contract=off"] + SAN + [str(drv), "-lm", "-o", str(exe)], check=True)
    r = _run(str(exe))
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.stdout.count("ok ") == 18


def test_sampler_under_sanitizers(tmp_path):
    if not _have("g++", "cpp", tmp_path):
        pytest.skip("g++ with ASan/UBSan not available")
    drv = tmp_path / "sampler_driver.cpp"
    drv.write_text(textwrap.dedent(SAMPLER_DRIVER))
    exe = tmp_path / "sampler_driver"
    csrc = os.path.join(ROOT, "paper_1705_04374_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-ffp-contract=off", "-I", os.path.join(ROOT, "include"), "-I", csrc]
                   + SAN + [os.path.join(csrc, "sampler.cpp"), str(drv), "-o", str(exe)], check=True)
    r = _run(str(exe))
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
