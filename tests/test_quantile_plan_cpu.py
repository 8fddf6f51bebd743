"""The host side of the quantile passes (cube_quantile_plan.h: ranks, pass
layouts, prefix tables, bin choice, interpolation), compiled with g++ under
AddressSanitizer and UBSan into a driver that runs the counting passes on
the CPU the way the kernel does.  Its results must equal the oracle's bit
for bit; every table and counter index is checked against its size.  No GPU
involved."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1111_6661_amd", "csrc")

DRIVER = r'''
#include "cube_quantile_plan.h"
#include <cstdio>
#include <cstdlib>
#include <vector>
using namespace cube;
#define CHECK(c) do { if (!(c)) { std::printf("FAIL line %d: %s\n", __LINE__, #c); std::exit(1); } } while (0)

static unsigned key_of(float v) {
    unsigned u; memcpy(&u, &v, 4);
    return u ^ ((unsigned)((int)u >> 31) | 0x80000000u);
}

// The counting passes on the CPU, voxel by voxel, as the kernel counts.
struct CpuPasses {
    std::vector<float> x;
    std::vector<unsigned long long> acc;
    int passes = 0, layout_bits = 0;
    int first(const unsigned long long **c, unsigned long long *nv) {
        acc.assign(QP_TOP, 0);
        unsigned long long n = 0;
        for (float v : x) {
            if (v != v) continue;
            ++n;
            acc[key_of(v) >> 20]++;
        }
        *c = acc.data();
        *nv = n;
        ++passes;
        return 0;
    }
    int refine(const QuantPassSpec &s, const unsigned char *tab, const unsigned long long **c) {
        CHECK(s.nl >= 1 && s.nl <= 3 && s.slots >= 1 && s.slots <= 128);
        CHECK(s.shift + s.width == 32 - 12 - (s.nl >= 2 ? s.w2 : 0) - (s.nl >= 3 ? s.w3 : 0));
        CHECK(((size_t)s.slots << s.width) <= 32768);           // the device counters
        CHECK(4096 + (size_t)s.t2_bytes + s.t3_bytes <= QP_TAB_MAX);
        // LDS of one block: histograms with the unused row 0, then the tables
        CHECK((((size_t)(s.slots + 1) << s.width) * 4 + 4096 + s.t2_bytes + s.t3_bytes)
              <= 160 * 1024 - 256);
        acc.assign((size_t)s.slots << s.width, 0);
        const unsigned char *t1 = tab, *t2 = tab + 4096, *t3 = t2 + s.t2_bytes;
        for (float v : x) {
            if (v != v) continue;
            const unsigned k = key_of(v);
            unsigned g = t1[k >> 20];
            if (s.nl >= 2) {
                const size_t i = ((size_t)g << s.w2) | ((k >> (20 - s.w2)) & ((1u << s.w2) - 1u));
                CHECK(i < (size_t)s.t2_bytes);
                g = t2[i];
            }
            if (s.nl >= 3) {
                const size_t i = ((size_t)g << s.w3) |
                                 ((k >> (20 - s.w2 - s.w3)) & ((1u << s.w3) - 1u));
                CHECK(i < (size_t)s.t3_bytes);
                g = t3[i];
            }
            if (g == 0) continue;
            CHECK(g <= (unsigned)s.slots);
            acc[((size_t)(g - 1) << s.width) | ((k >> s.shift) & ((1u << s.width) - 1u))]++;
        }
        *c = acc.data();
        ++passes;
        layout_bits = layout_bits * 100 + s.width;
        return 0;
    }
};

int main(int argc, char **argv) {
    CHECK(argc == 3);
    CpuPasses P;
    FILE *f = std::fopen(argv[1], "rb");
    CHECK(f);
    float v;
    while (std::fread(&v, 4, 1, f) == 1) P.x.push_back(v);
    std::fclose(f);
    std::vector<double> q;
    f = std::fopen(argv[2], "rb");
    CHECK(f);
    double d;
    while (std::fread(&d, 8, 1, f) == 1) q.push_back(d);
    std::fclose(f);
    std::vector<unsigned char> tab(QP_TAB_MAX);
    std::vector<double> out(q.size());
    uint64_t nv = 0;
    const int rc = quantiles_run(P, q.data(), (int)q.size(), out.data(), &nv, tab.data(), 7);
    std::printf("rc %d n %llu passes %d layout %d\n", rc, (unsigned long long)nv, P.passes,
                P.layout_bits);
    for (double o : out) {
        unsigned long long u; memcpy(&u, &o, 8);
        std::printf("%016llx\n", u);
    }
    return 0;
}
'''


@pytest.fixture(scope="module")
def driver():
    d = tempfile.mkdtemp(prefix="qplan_")
    src = os.path.join(d, "qplan.cpp")
    exe = os.path.join(d, "qplan")
    with open(src, "w") as f:
        f.write(DRIVER)
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-I", CSRC, "-o", exe, src])
    yield exe, d


def run(driver, a, levels):
    exe, d = driver
    a = np.ascontiguousarray(a, dtype=np.float32).reshape(-1)
    lv = np.ascontiguousarray(levels, dtype=np.float64)
    fa, fq = os.path.join(d, "a.bin"), os.path.join(d, "q.bin")
    a.tofile(fa)
    lv.tofile(fq)
    r = subprocess.run([exe, fa, fq], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = r.stdout.split("\n")
    head = lines[0].split()
    rc, n, passes, layout = int(head[1]), int(head[3]), int(head[5]), int(head[7])
    vals = np.array([int(x, 16) for x in lines[1:1 + lv.size]], dtype=np.uint64).view(np.float64)
    return rc, n, passes, layout, vals


def check(driver, a, levels, layout=None):
    rc, n, passes, got_layout, vals = run(driver, a, levels)
    assert rc == 0 and n == int(np.count_nonzero(~np.isnan(a)))
    want = oracle.quantiles(a, levels)
    assert np.array_equal(vals.view(np.uint64), want.view(np.uint64)), (levels, vals, want)
    if layout is not None:
        assert got_layout == layout, got_layout
    return passes


def test_random_levels(driver):
    rng = np.random.default_rng(1)
    a = (rng.standard_normal(60_000) * 3 + 1).astype(np.float32)
    a[rng.random(a.size) < 0.02] = np.nan
    assert check(driver, a, [0.25, 0.5, 0.75], layout=1208) == 3
    check(driver, a, np.concatenate([[0.0, 1.0, 1e-12, 1 - 1e-12], rng.random(60)]))


def test_many_buckets_take_four_passes(driver):
    rng = np.random.default_rng(2)
    a = np.concatenate([2.0 ** e * (1 + 0.1 * rng.random(500)) for e in range(-40, 40)])
    a = np.concatenate([a, -a[:3000]]).astype(np.float32)
    rng.shuffle(a)
    assert check(driver, a, np.linspace(0, 1, 64), layout=80606) == 4


def test_many_ranks_in_few_buckets(driver):
    rng = np.random.default_rng(3)
    a = np.concatenate([2.0 ** e * (1 + 0.1 * rng.random(20_000)) for e in (0, 5)]).astype(np.float32)
    check(driver, a, np.sort(rng.random(64)), layout=80606)   # 128 ranks > 96
    check(driver, a, np.sort(rng.random(40)), layout=1208)    # 80 ranks, 2 buckets


def test_special_values_ties_and_tiny(driver):
    a = np.array([0.0, -0.0, np.nan, np.inf, -np.inf, 0.0, 3.5, -1e-45, 1e-45, 3.5, 3.5, -2.0],
                 dtype=np.float32)
    check(driver, a, np.linspace(0, 1, 33))
    check(driver, np.array([7.0], np.float32), [0.0, 0.5, 1.0])
    check(driver, np.array([2.0, -1.0], np.float32), [0.0, 0.3, 1.0])
    check(driver, np.round(np.random.default_rng(4).standard_normal(5000)).astype(np.float32),
          np.linspace(0, 1, 64))


def test_no_valid_voxel(driver):
    rc, n, passes, _, _ = run(driver, np.full(10, np.nan, np.float32), [0.5])
    assert rc == 7 and n == 0 and passes == 1
