// cube_quantile_plan.h -- the host side of the quantile passes: which ranks
// the levels need, the order of the key bits over the passes, the prefix
// tables each pass reads, the choice of each rank's bin from the counts, and
// the interpolation of the levels.  Plain C++ with no GPU calls: the caller
// supplies the passes themselves (QuantPasses below).
//
// The key of a float orders like its value (-0 before +0).  Pass 0 counts
// the top 12 key bits of every valid voxel.  Then, when the ranks fall in at
// most 8 distinct top buckets and number at most 96, two passes refine them
// by 12 and 8 more bits; otherwise three passes by 8, 6 and 6 bits.  A pass
// after the first counts, for every wanted prefix of `done` bits, the next
// `width` bits of the voxels under it.  It finds a voxel's prefix through a
// chain of byte tables, one per level of the prefix (widths 12, then w2,
// then w3): entries hold the prefix's index + 1 (0: none), row 0 of every
// further table is all zero, and a voxel whose chain ends at 0 is not
// counted.
#pragma once

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

namespace cube {

constexpr int QP_TOP = 4096;                       // bins of the first pass
constexpr size_t QP_TAB_MAX = 4096 + 9 * 4096 + 129 * 64;  // table bytes at most

// One refinement pass as the caller runs it.
struct QuantPassSpec {
    int nl;                  // prefix levels (1..3)
    int shift, width;        // count key bits [shift, shift + width)
    int w2, w3;              // widths of the second and third prefix levels
    int slots;               // wanted prefixes: rows of counts, 1 << width each
    int t2_bytes, t3_bytes;  // table sizes after the 4096-byte first table
};

// A rank being refined: the key bits found so far (at the top of `key`) and
// the rank left inside that prefix.
struct QuantWant {
    unsigned long long rank;
    unsigned int key;
};

// The bin of `h` (nbins counters) holding rank r; r becomes the rank inside
// that bin.  The counts sum to more than r when they come from a pass over
// the same data.
inline unsigned int qp_pick_bin(const unsigned long long *h, int nbins, unsigned long long &r)
{
    int b = 0;
    while (b < nbins - 1 && h[b] <= r) r -= h[b++];
    return (unsigned int)b;
}

inline float qp_key_to_float(unsigned int k)
{
    const unsigned int u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

// a + f (b - a) between the voxels of two neighbouring ranks; equal ends
// give a, an infinite end is the result, -Inf to +Inf is NaN.
inline double qp_interpolate(double a, double b, double f)
{
    if (a == b) return a;
    if (isinf(a) && isinf(b)) return NAN;
    if (isinf(a)) return a;
    if (isinf(b)) return b;
    return a + f * (b - a);
}

// The distinct values of the top `bits` key bits among the wanted ranks,
// ascending.
inline std::vector<unsigned int> qp_prefixes(const std::vector<QuantWant> &want, int bits)
{
    std::vector<unsigned int> p;
    for (const QuantWant &x : want) p.push_back(x.key >> (32 - bits));
    std::sort(p.begin(), p.end());
    p.erase(std::unique(p.begin(), p.end()), p.end());
    return p;
}

template <class T>
inline size_t qp_index(const std::vector<T> &p, T v)
{
    return (size_t)(std::lower_bound(p.begin(), p.end(), v) - p.begin());
}

// The ranks levels q[0..m-1] need among n valid voxels, ascending and
// distinct: floor(q (n - 1)) and, when q (n - 1) is not whole, the next.
inline std::vector<unsigned long long> qp_ranks(const double *q, int m, unsigned long long n)
{
    std::vector<unsigned long long> r;
    for (int i = 0; i < m; ++i) {
        const double h = q[i] * (double)(n - 1);
        const double j = floor(h);
        r.push_back((unsigned long long)j);
        if (h - j > 0.0) r.push_back((unsigned long long)j + 1);
    }
    std::sort(r.begin(), r.end());
    r.erase(std::unique(r.begin(), r.end()), r.end());
    return r;
}

// Fill the tables of a pass with `nl` prefix levels (widths 12, lev[1],
// lev[2]) into tab (QP_TAB_MAX bytes); returns the pass's prefixes (its
// histogram rows are their indices + 1) and sets the table sizes.
inline std::vector<unsigned int> qp_tables(const std::vector<QuantWant> &want, int nl,
                                           const int (&lev)[3], unsigned char *tab,
                                           int *t2_bytes, int *t3_bytes)
{
    unsigned char *t1 = tab;
    memset(t1, 0, QP_TOP);
    const std::vector<unsigned int> p1 = qp_prefixes(want, 12);
    for (size_t i = 0; i < p1.size(); ++i) t1[p1[i]] = (unsigned char)(i + 1);
    *t2_bytes = *t3_bytes = 0;
    if (nl < 2) return p1;
    const std::vector<unsigned int> p2 = qp_prefixes(want, 12 + lev[1]);
    unsigned char *t2 = t1 + QP_TOP;
    *t2_bytes = (int)((p1.size() + 1) << lev[1]);
    memset(t2, 0, (size_t)*t2_bytes);
    for (size_t i = 0; i < p2.size(); ++i) {
        const unsigned int up = (unsigned int)qp_index(p1, p2[i] >> lev[1]) + 1;
        t2[(up << lev[1]) | (p2[i] & ((1u << lev[1]) - 1u))] = (unsigned char)(i + 1);
    }
    if (nl < 3) return p2;
    const std::vector<unsigned int> p3 = qp_prefixes(want, 12 + lev[1] + lev[2]);
    unsigned char *t3 = t2 + *t2_bytes;
    *t3_bytes = (int)((p2.size() + 1) << lev[2]);
    memset(t3, 0, (size_t)*t3_bytes);
    for (size_t i = 0; i < p3.size(); ++i) {
        const unsigned int up = (unsigned int)qp_index(p2, p3[i] >> lev[2]) + 1;
        t3[(up << lev[2]) | (p3[i] & ((1u << lev[2]) - 1u))] = (unsigned char)(i + 1);
    }
    return p3;
}

// The passes as the caller provides them:
//   int first(const unsigned long long **counts, unsigned long long *n_valid)
//       counts the top 12 key bits of the valid voxels (QP_TOP counters);
//   int refine(const QuantPassSpec &, const unsigned char *tab,
//              const unsigned long long **counts)
//       one refinement pass (spec.slots << spec.width counters).
// Each returns 0 or an error code, which quantiles_run returns as it is.
// Levels q[0..m-1] (each in [0, 1], at most 64 of them) give out[0..m-1];
// *n_valid is set after the first pass; `no_valid` is returned when there
// is no valid voxel.
template <class Passes>
int quantiles_run(Passes &passes, const double *q, int m, double *out, uint64_t *n_valid,
                  unsigned char *tab, int no_valid)
{
    const unsigned long long *h = nullptr;
    unsigned long long n = 0;
    int rc = passes.first(&h, &n);
    if (rc) return rc;
    if (n_valid) *n_valid = n;
    if (n == 0) return no_valid;

    const std::vector<unsigned long long> ranks = qp_ranks(q, m, n);
    std::vector<QuantWant> want(ranks.size());
    for (size_t i = 0; i < ranks.size(); ++i) {
        want[i].rank = ranks[i];
        want[i].key = qp_pick_bin(h, QP_TOP, want[i].rank) << 20;
    }

    const bool wide = qp_prefixes(want, 12).size() <= 8 && want.size() <= 96;
    static const int wide_w[] = {12, 8}, narrow_w[] = {8, 6, 6};
    const int *widths = wide ? wide_w : narrow_w;
    const int npass = wide ? 2 : 3;
    int lev[3] = {12, 0, 0};  // widths of the prefix levels
    int done = 12;            // key bits found so far
    for (int p = 0; p < npass; ++p) {
        QuantPassSpec s;
        s.nl = p + 1;
        s.width = widths[p];
        s.shift = 32 - done - s.width;
        s.w2 = lev[1];
        s.w3 = lev[2];
        const std::vector<unsigned int> pre = qp_tables(want, s.nl, lev, tab, &s.t2_bytes,
                                                        &s.t3_bytes);
        s.slots = (int)pre.size();
        if ((rc = passes.refine(s, tab, &h))) return rc;
        for (QuantWant &x : want) {
            const size_t slot = qp_index(pre, x.key >> (32 - done));
            const unsigned int b = qp_pick_bin(h + (slot << s.width), 1 << s.width, x.rank);
            x.key |= b << s.shift;
        }
        if (s.nl < 3) lev[s.nl] = s.width;
        done += s.width;
    }

    for (int i = 0; i < m; ++i) {
        const double hh = q[i] * (double)(n - 1);
        const double j = floor(hh);
        const double f = hh - j;
        const double a = qp_key_to_float(want[qp_index(ranks, (unsigned long long)j)].key);
        const double b =
            f > 0.0 ? qp_key_to_float(want[qp_index(ranks, (unsigned long long)j + 1)].key) : a;
        out[i] = qp_interpolate(a, b, f);
    }
    return 0;
}

}  // namespace cube
