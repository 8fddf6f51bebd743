"""The server's admission and batching policy (cube_policy.h), compiled with
g++ into a small test driver: no GPU involved."""
import os
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1111_6661_amd", "csrc")

DRIVER = r'''
#include "cube_policy.h"
#include <cstdio>
#include <cstdlib>
using namespace cube;
#define CHECK(c) do { if (!(c)) { std::printf("FAIL line %d: %s\n", __LINE__, #c); std::exit(1); } } while (0)
int main() {
    std::vector<PolicyQuery> b;
    {   // batches take the oldest queries, up to max_batch
        PolicyLimits L; L.slots = 2; L.max_batch = 3; L.max_inflight_bytes = 1000;
        Policy p(L);
        for (uint64_t i = 1; i <= 7; ++i) CHECK(p.submit({i, 10, 10}));
        int s0 = p.next_batch(b); CHECK(s0 == 0 && b.size() == 3 && b[0].id == 1 && b[2].id == 3);
        int s1 = p.next_batch(b); CHECK(s1 == 1 && b.size() == 3 && b[0].id == 4);
        CHECK(p.next_batch(b) == -1);          // no free slot
        CHECK(p.busy_slots() == 2 && p.waiting() == 1 && p.inflight_bytes() == 60);
        p.complete(s0);                        // a slot frees: the rest is admitted
        int s2 = p.next_batch(b); CHECK(s2 == 0 && b.size() == 1 && b[0].id == 7);
        p.complete(s1); p.complete(s2);
        CHECK(p.inflight_bytes() == 0 && p.busy_slots() == 0);
        p.complete(5); p.complete(-1);         // out-of-range slots are ignored
    }
    {   // admission by memory: a batch stops at the byte budget
        PolicyLimits L; L.slots = 4; L.max_batch = 100; L.max_inflight_bytes = 100;
        Policy p(L);
        for (uint64_t i = 1; i <= 5; ++i) CHECK(p.submit({i, 1, 40}));
        int s0 = p.next_batch(b); CHECK(s0 >= 0 && b.size() == 2);   // 80 of 100
        CHECK(p.next_batch(b) == -1);          // 40 more would exceed the budget
        p.complete(s0);
        CHECK(p.next_batch(b) >= 0 && b.size() == 2);
    }
    {   // a query larger than the budget runs alone when the device is idle
        PolicyLimits L; L.slots = 2; L.max_batch = 8; L.max_inflight_bytes = 100;
        Policy p(L);
        CHECK(p.submit({1, 1, 50})); CHECK(p.submit({2, 1, 500})); CHECK(p.submit({3, 1, 10}));
        int s0 = p.next_batch(b); CHECK(b.size() == 1 && b[0].id == 1);
        CHECK(p.next_batch(b) == -1);          // the big one waits for an idle device
        p.complete(s0);
        int s1 = p.next_batch(b); CHECK(s1 >= 0 && b.size() == 1 && b[0].id == 2);
        CHECK(p.next_batch(b) == -1);          // nothing fits beside it
        p.complete(s1);
        CHECK(p.next_batch(b) >= 0 && b[0].id == 3);
    }
    {   // voxel limit per batch, queue limit
        PolicyLimits L; L.slots = 1; L.max_batch = 10; L.max_batch_voxels = 100; L.max_queue = 3;
        Policy p(L);
        CHECK(p.submit({1, 60, 1})); CHECK(p.submit({2, 60, 1})); CHECK(p.submit({3, 30, 1}));
        CHECK(!p.submit({4, 1, 1}));           // queue full
        CHECK(p.next_batch(b) == 0 && b.size() == 1);  // 60 + 60 > 100
        p.complete(0);
        CHECK(p.next_batch(b) == 0 && b.size() == 2);  // 60 + 30
    }
    std::printf("policy ok\n");
    return 0;
}
'''


def test_policy_driver():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "policy_test.cpp")
        exe = os.path.join(d, "policy_test")
        with open(src, "w") as f:
            f.write(DRIVER)
        subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-fsanitize=address,undefined",
                               "-I", CSRC, "-o", exe, src])
        r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "policy ok" in r.stdout
