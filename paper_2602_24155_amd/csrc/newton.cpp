// Newton-polygon invariants of the integer L-polynomial (host only):
// cr_newton_polygon of include/crfrob.h.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/crfrob.h"
#include "host.hpp"

namespace crf {
void set_last_error(const std::string &msg);
}

namespace {

using crf::binom;
using crf::count_monomials;

// |x| of a signed 256-bit two's-complement integer (4 little-endian words),
// divided by p as long as the remainder is zero: the p-adic valuation.
int valuation256(const int64_t *w, int p, bool &zero) {
    uint64_t m[4];
    for (int k = 0; k < 4; k++) m[k] = (uint64_t)w[k];
    if ((int64_t)m[3] < 0) {  // negate
        unsigned carry = 1;
        for (int k = 0; k < 4; k++) {
            const uint64_t v = ~m[k] + carry;
            carry = carry && v == 0;
            m[k] = v;
        }
    }
    zero = (m[0] | m[1] | m[2] | m[3]) == 0;
    if (zero) return 0;
    int v = 0;
    for (;;) {
        uint64_t q[4];
        unsigned __int128 r = 0;
        for (int k = 3; k >= 0; k--) {
            const unsigned __int128 cur = (r << 64) | m[k];
            q[k] = (uint64_t)(cur / (unsigned)p);
            r = cur % (unsigned)p;
        }
        if (r != 0) return v;
        std::memcpy(m, q, sizeof(m));
        v++;
    }
}

long long hodge_count(int nv, int d, int m) {
    const int n = nv - 1, k = d * m - n - 1;
    long long h = 0;
    for (int j = 0; j < nv; j++) {
        const int kk = k - j * (d - 1);
        if (kk < 0) break;
        h += ((j & 1) ? -1 : 1) * binom(nv, j) * count_monomials(nv, kk);
    }
    return h;
}

// height of the polygon with the given vertices at abscissa x, as num / den
// (den = length of the segment containing x)
void value_at(const std::vector<std::pair<int, long long>> &v, int x, long long &num, long long &den) {
    for (size_t k = 0; k + 1 < v.size(); k++) {
        const int x1 = v[k].first, x2 = v[k + 1].first;
        if (x >= x1 && x <= x2) {
            den = x2 - x1;
            num = v[k].second * den + (v[k + 1].second - v[k].second) * (x - x1);
            return;
        }
    }
    num = v.back().second;
    den = 1;
}

}  // namespace

extern "C" cr_status cr_newton_polygon(int32_t nvars, int32_t degree, int32_t p, const int64_t *lpoly,
                                       cr_newton *out) {
    if (!lpoly || !out || nvars < 3 || nvars > 6 || degree < 2 || p < 2) {
        crf::set_last_error("cr_newton_polygon: bad arguments");
        return CR_EINVAL;
    }
    const int n = nvars - 1, w = n - 1;
    std::vector<long long> hod(n + 1, 0);
    int b = 0;
    for (int m = 1; m <= n; m++) b += (int)(hod[m] = hodge_count(nvars, degree, m));
    if (b < 1 || b >= CR_NEWTON_MAX) {
        crf::set_last_error("cr_newton_polygon: basis size out of range");
        return CR_EINVAL;
    }
    // points (j, v_p(a_j)) of the nonzero coefficients; a_0 must be 1
    std::vector<std::pair<int, long long>> pts;
    for (int j = 0; j <= b; j++) {
        bool zero = false;
        const int v = valuation256(lpoly + 4 * (size_t)j, p, zero);
        if (!zero) pts.push_back({j, v});
    }
    if (pts.empty() || pts.front().first != 0 || pts.front().second != 0 || pts.back().first != b) {
        crf::set_last_error("cr_newton_polygon: Q(T) must have a_0 = 1 and degree b");
        return CR_EINVAL;
    }
    // lower convex hull (left to right)
    std::vector<std::pair<int, long long>> hull;
    for (const auto &q : pts) {
        while (hull.size() >= 2) {
            const auto &a = hull[hull.size() - 2], &c = hull.back();
            if ((c.second - a.second) * (long long)(q.first - a.first) >=
                (q.second - a.second) * (long long)(c.first - a.first))
                hull.pop_back();
            else
                break;
        }
        hull.push_back(q);
    }
    // merge collinear runs into segments of one slope
    std::vector<std::pair<int, long long>> seg;  // (length, rise)
    for (size_t k = 0; k + 1 < hull.size(); k++) {
        const int len = hull[k + 1].first - hull[k].first;
        const long long rise = hull[k + 1].second - hull[k].second;
        if (!seg.empty() && seg.back().second * len == rise * seg.back().first) {
            seg.back().first += len;
            seg.back().second += rise;
        } else {
            seg.push_back({len, rise});
        }
    }
    // Hodge polygon: slope n - m with multiplicity h_m, ascending
    std::vector<std::pair<int, long long>> hv{{0, 0}}, nv_{{0, 0}};
    std::vector<std::pair<int, int>> hseg;  // (length, slope)
    for (int m = n; m >= 1; m--)
        if (hod[m] > 0) {
            hseg.push_back({(int)hod[m], n - m});
            hv.push_back({hv.back().first + (int)hod[m], hv.back().second + hod[m] * (n - m)});
        }
    for (const auto &sg : seg) nv_.push_back({nv_.back().first + sg.first, nv_.back().second + sg.second});
    std::memset(out, 0, sizeof(*out));
    out->b = b;
    out->nseg = (int)seg.size();
    for (size_t k = 0; k < seg.size(); k++) {
        out->seg_len[k] = seg[k].first;
        out->seg_rise[k] = (int32_t)seg[k].second;
    }
    // p-rank: the Newton segment of the smallest Hodge slope
    const int smin = hseg.front().second;
    for (const auto &sg : seg)
        if (sg.second == (long long)smin * sg.first) out->p_rank += sg.first;
    out->ordinary = 1;
    for (int x = 0; x <= b && out->ordinary; x++) {
        long long a, da, c, dc;
        value_at(nv_, x, a, da);
        value_at(hv, x, c, dc);
        if (a * dc != c * da) out->ordinary = 0;
    }
    out->supersingular = seg.size() == 1 && 2 * seg[0].second == (long long)w * seg[0].first;
    // height: Hodge numbers 1, b - 2, 1 at slopes w/2 - 1, w/2, w/2 + 1 (even w); first
    // Newton slope w/2 - 1/h
    out->height = -1;
    if (w % 2 == 0 && hseg.size() == 3 && hseg[0].first == 1 && hseg[2].first == 1 && hseg[1].second == w / 2 &&
        hseg[0].second == w / 2 - 1) {
        const long long len = seg[0].first, rise = seg[0].second;
        if (rise * 2 == (long long)w * len) {
            out->height = 0;  // supersingular
        } else {
            // w/2 - rise/len = 1/h  <=>  h = len / (w/2 len - rise)
            const long long den = (long long)(w / 2) * len - rise;
            out->height = (den > 0 && len % den == 0) ? (int32_t)(len / den) : -1;
        }
    }
    // domino number of a surface: min (Newton - Hodge) over the slope-1 part of the Hodge polygon
    out->domino_num = -1;
    out->domino_den = 1;
    if (n == 3) {
        int x0 = 0, x1 = 0;
        for (const auto &h : hseg) {
            if (h.second < 1) x0 += h.first;
            if (h.second <= 1) x1 += h.first;
        }
        bool first = true;
        for (int x = x0; x <= x1; x++) {
            long long a, da, c, dc;
            value_at(nv_, x, a, da);
            value_at(hv, x, c, dc);
            // (a / da) - (c / dc)
            long long num = a * dc - c * da, den = da * dc;
            const long long g = std::__gcd(num < 0 ? -num : num, den);
            if (g > 1) {
                num /= g;
                den /= g;
            }
            if (first || num * out->domino_den < (long long)out->domino_num * den) {
                out->domino_num = (int32_t)num;
                out->domino_den = (int32_t)den;
                first = false;
            }
        }
    }
    return CR_OK;
}
