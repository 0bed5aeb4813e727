"""The C interface's host code built with AddressSanitizer (leak detection
on) and driven through its validation paths and, where no GPU is visible,
through its HIP-failure paths (every launch and allocation fails there):
an out-of-bounds access or a leak on an error path aborts the driver.  The
device code is built as usual; the sanitizer applies to the host side only.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2411_13532_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

DRIVER = r"""
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include "ttm.h"

#define CHECK(x, want) do { const int r_ = (x); if (r_ != (want)) { \
    std::fprintf(stderr, "line %d: %s = %d, want %d\n", __LINE__, #x, r_, int(want)); return 1; } } while (0)
static void *fake(int k) { return reinterpret_cast<void *>((uintptr_t(1) << 40) + (uintptr_t(k) << 32)); }
static void *at(int k, uintptr_t off) { return reinterpret_cast<char *>(fake(k)) + off; }

static int validation() {
    if (!ttm_status_string(TTM_ERR_HIP) || ttm_version() < 10000) return 1;
    CHECK(ttm_set_slab_kernel(7), TTM_ERR_INVALID_ARG);
    CHECK(ttm_set_slab_kernel(0), TTM_OK);
    CHECK(ttm_chain_supported(TTM_BF16, TTM_F32, TTM_F32, TTM_MATH_BF16X3), 1);
    CHECK(ttm_chain_supported(TTM_F64, TTM_F32, TTM_F32, TTM_MATH_F32), 0);
    ttm_shape s = {{8, 8, 8}, {4, 4, 4}}, bad = {{0, 8, 8}, {4, 4, 4}};
    if (ttm_chain_workspace_size(&s, TTM_F32, TTM_MATH_F32) == 0) return 1;
    if (ttm_chain_workspace_size(&bad, TTM_F32, TTM_MATH_F32) != 0) return 1;
    const size_t ws = size_t(1) << 30;
    CHECK(ttm_chain(nullptr, fake(0), TTM_F32, fake(1), fake(2), fake(3), TTM_F32, fake(4), TTM_F32, TTM_MATH_F32,
                    fake(5), ws, nullptr), TTM_ERR_INVALID_ARG);
    CHECK(ttm_chain(&bad, fake(0), TTM_F32, fake(1), fake(2), fake(3), TTM_F32, fake(4), TTM_F32, TTM_MATH_F32,
                    fake(5), ws, nullptr), TTM_ERR_INVALID_ARG);
    CHECK(ttm_chain(&s, at(0, 4), TTM_F32, fake(1), fake(2), fake(3), TTM_F32, fake(4), TTM_F32, TTM_MATH_F32,
                    fake(5), ws, nullptr), TTM_ERR_INVALID_ARG);
    CHECK(ttm_chain(&s, fake(0), TTM_F32, fake(1), fake(2), fake(3), TTM_F32, fake(4), TTM_BF16, TTM_MATH_F32,
                    fake(5), ws, nullptr), TTM_ERR_UNSUPPORTED);
    CHECK(ttm_chain(&s, fake(0), TTM_F32, fake(1), fake(2), fake(3), TTM_F32, fake(4), TTM_F32, TTM_MATH_F32,
                    fake(5), 16, nullptr), TTM_ERR_WORKSPACE);
    CHECK(ttm_chain(&s, fake(0), TTM_F32, fake(1), fake(2), fake(3), TTM_F32, at(0, 256), TTM_F32, TTM_MATH_F32,
                    fake(5), ws, nullptr), TTM_ERR_ALIAS);
    CHECK(ttm_chain_noalloc(&s, fake(0), TTM_F32, fake(1), fake(2), fake(3), TTM_F32, at(0, 256), TTM_F32,
                            TTM_MATH_F32, nullptr), TTM_ERR_ALIAS);
    CHECK(ttm_chain_backward(&s, fake(0), fake(1), fake(2), fake(3), fake(4), TTM_F32, nullptr, nullptr, nullptr,
                             nullptr, TTM_MATH_F32, fake(9), ws, nullptr), TTM_ERR_INVALID_ARG);
    CHECK(ttm_chain_backward(&s, fake(0), fake(1), fake(2), fake(3), fake(4), TTM_F32, fake(1), fake(6), fake(7),
                             fake(8), TTM_MATH_F32, fake(9), ws, nullptr), TTM_ERR_ALIAS);
    int64_t dims[18] = {3, 4, 5, 2, 3, 6, 1, 1, 1, 1, 1, 1, 4, 2, 17, 5, 1, 2};
    ttm_batched_plan *p = nullptr;
    CHECK(ttm_batched_plan_create(3, dims, TTM_F32, TTM_MATH_F32, nullptr, nullptr, &p), TTM_ERR_INVALID_ARG);
    CHECK(ttm_batched_plan_create(0, dims, TTM_F32, TTM_MATH_F32, nullptr, nullptr, &p), TTM_ERR_INVALID_ARG);
    CHECK(ttm_batched_plan_create(3, dims, TTM_F32, TTM_MATH_BF16, nullptr, nullptr, &p), TTM_ERR_UNSUPPORTED);
    if (p) return 1;
    CHECK(ttm_batched_plan_destroy(nullptr), TTM_ERR_INVALID_ARG);
    CHECK(ttm_batched_plan_set_config(nullptr, 256, 1, 1, nullptr), TTM_ERR_INVALID_ARG);
    const int64_t cd[3] = {8, 16, 32};
    const ttm_compact_coef coef = {1.0 / 3.0, 14.0 / 9.0, 1.0 / 9.0, 0.1}, nodom = {0.5, 14.0 / 9.0, 1.0 / 9.0, 0.1};
    const size_t cws = ttm_compact_workspace_size(16, TTM_F64);
    CHECK(ttm_compact_apply(cd, 0, fake(0), fake(1), TTM_F64, &coef, fake(2), cws, 0, nullptr), TTM_ERR_INVALID_ARG);
    CHECK(ttm_compact_apply(cd, 2, fake(0), fake(1), TTM_F64, &nodom, fake(2), cws, 0, nullptr), TTM_ERR_INVALID_ARG);
    CHECK(ttm_compact_apply(cd, 2, fake(0), at(0, 800), TTM_F64, &coef, fake(2), cws, 0, nullptr), TTM_ERR_ALIAS);
    ttm_shape hs = {{129, 4, 4}, {4, 4, 4}};
    if (ttm_hosvd_workspace_size(&hs) != 0) return 1;
    const int perm_bad[3] = {0, 0, 2};
    CHECK(ttm_reorder(cd, perm_bad, fake(0), fake(1), TTM_F64, 0, nullptr), TTM_ERR_INVALID_ARG);
    char names[4 * 64];
    int64_t counts[4];
    double ms[4];
    CHECK(ttm_timing_enable(0), TTM_OK);
    if (ttm_timing_collect(names, counts, ms, 4) < 0) return 1;
    return 0;
}

// every HIP call fails where no GPU is visible: valid requests must come back
// as TTM_ERR_HIP, hand out no plan, and leave nothing allocated behind
static int hip_failures() {
    ttm_shape s = {{64, 300, 128}, {16, 20, 40}};
    const int maths[4] = {TTM_MATH_F64, TTM_MATH_F32, TTM_MATH_BF16, TTM_MATH_BF16X3};
    for (int m : maths) {
        const int fdt = m == TTM_MATH_F64 ? TTM_F64 : TTM_F32;
        const int xdt = (m == TTM_MATH_BF16 || m == TTM_MATH_BF16X3) ? TTM_BF16 : fdt;
        const size_t ws = ttm_chain_workspace_size(&s, xdt, m);
        CHECK(ttm_chain(&s, fake(0), xdt, fake(1), fake(2), fake(3), fdt, fake(4), fdt, m, fake(5), ws, nullptr),
              TTM_ERR_HIP);
    }
    ttm_shape b = {{32, 64, 64}, {8, 8, 8}};
    const size_t bws = ttm_chain_backward_workspace_size(&b, TTM_F32, TTM_MATH_F32);
    CHECK(ttm_chain_backward(&b, fake(0), fake(1), fake(2), fake(3), fake(4), TTM_F32, fake(5), fake(6), fake(7),
                             fake(8), TTM_MATH_F32, fake(9), bws, nullptr), TTM_ERR_HIP);
    CHECK(ttm_stream_copy(fake(0), fake(1), 4096, nullptr), TTM_ERR_HIP);
    int64_t dims[24];
    for (int k = 0; k < 4; ++k)
        for (int i = 0; i < 6; ++i) dims[6 * k + i] = 5 + i % 3;
    for (int r = 0; r < 20; ++r) {
        ttm_batched_plan *p = reinterpret_cast<ttm_batched_plan *>(uintptr_t(1234));
        CHECK(ttm_batched_plan_create(4, dims, TTM_F32, TTM_MATH_F32, nullptr, nullptr, &p), TTM_ERR_HIP);
        if (p) return 1;
    }
    const int64_t cd[3] = {8, 16, 32};
    const ttm_compact_coef coef = {1.0 / 3.0, 14.0 / 9.0, 1.0 / 9.0, 0.1};
    CHECK(ttm_compact_apply(cd, 2, fake(0), fake(1), TTM_F64, &coef, fake(2),
                            ttm_compact_workspace_size(16, TTM_F64), 0, nullptr), TTM_ERR_HIP);
    const int perm[3] = {2, 0, 1};
    CHECK(ttm_reorder(cd, perm, fake(0), fake(1), TTM_F64, 0, nullptr), TTM_ERR_HIP);
    ttm_shape hs = {{16, 12, 10}, {4, 3, 2}};
    CHECK(ttm_hosvd(&hs, fake(0), fake(1), fake(2), fake(3), nullptr, fake(4), ttm_hosvd_workspace_size(&hs), nullptr),
          TTM_ERR_HIP);
    return 0;
}

int main(int argc, char **argv) {
    if (validation()) return 1;
    if (argc > 1 && std::strcmp(argv[1], "nogpu") == 0 && hip_failures()) return 1;
    std::printf("C interface under AddressSanitizer: ok\n");
    return 0;
}
"""


def _no_gpu():
    try:
        import torch
        return not torch.cuda.is_available()
    except Exception:
        return True


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="needs hipcc")
def test_c_interface_under_address_sanitizer(tmp_path):
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    flags = ["-std=c++17", "-O1", "-g", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
             f"-I{INCLUDE}", "-w"]
    drv = tmp_path / "driver.cpp"
    drv.write_text(DRIVER)
    units = srcs + [str(drv)]
    objs = [str(tmp_path / (os.path.basename(u) + ".o")) for u in units]
    jobs = max(1, min(8, os.cpu_count() or 1))
    pending = list(zip(units, objs))
    running = []
    while pending or running:
        while pending and len(running) < jobs:
            u, o = pending.pop(0)
            running.append((u, subprocess.Popen([HIPCC, *flags, "-c", u, "-o", o], stdout=subprocess.PIPE,
                                                stderr=subprocess.STDOUT)))
        u, proc = running.pop(0)
        out, _ = proc.communicate()
        assert proc.returncode == 0, f"{u}: {out.decode(errors='replace')[-3000:]}"
    exe = str(tmp_path / "driver")
    link = subprocess.run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", *objs, "-o", exe],
                          capture_output=True, text=True)
    assert link.returncode == 0, link.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0")
    args = [exe] + (["nogpu"] if _no_gpu() else [])
    r = subprocess.run(args, capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-6000:]
    assert "C interface under AddressSanitizer: ok" in r.stdout
