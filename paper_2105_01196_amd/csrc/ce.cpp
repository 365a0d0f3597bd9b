// Clustering error (CE, Sec. 2.2, Eq. 1) between detected biclusters and the
// ground truth, for scoring recovery of planted biclusters. Host code.
//
// A bicluster is the product of a row set and a column set, so the cells two
// biclusters share number |rows ∩ rows'| * |cols ∩ cols'|: that is the
// confusion matrix. D_max is the largest total of a one-to-one assignment
// between the two sets (Munkres' algorithm, here the shortest augmenting
// path form with potentials, O(n^3)); U collects every cell covered by any
// bicluster of either set.
#include <algorithm>
#include <cstdint>
#include <limits>
#include <vector>

#include "internal.h"

namespace ebic {
namespace {

struct Bic {
    std::vector<int32_t> rows, cols;  // sorted, distinct
};

int64_t shared(const std::vector<int32_t> &a, const std::vector<int32_t> &b) {
    int64_t n = 0;
    size_t i = 0, j = 0;
    while (i < a.size() && j < b.size()) {
        if (a[i] < b[j]) {
            i++;
        } else if (b[j] < a[i]) {
            j++;
        } else {
            n++;
            i++;
            j++;
        }
    }
    return n;
}

// Largest total of a one-to-one assignment of rows to columns of the n x m
// profit matrix w (row-major); rows or columns left over stay unassigned.
// The square cost matrix max(w) - w (zero-padded to max(n, m)) is solved for
// its minimum with row and column potentials, adding one row at a time
// along a shortest augmenting path.
int64_t max_assignment(const std::vector<int64_t> &w, int n, int m) {
    const int s = std::max(n, m);
    if (s == 0) return 0;
    int64_t top = 0;
    for (int64_t v : w) top = std::max(top, v);
    auto cost = [&](int i, int j) -> int64_t {
        const int64_t v = (i < n && j < m) ? w[(size_t)i * m + j] : 0;
        return top - v;
    };
    const int64_t INF = std::numeric_limits<int64_t>::max() / 4;
    // 1-based: column 0 is the virtual start of each augmenting path
    std::vector<int64_t> u(s + 1, 0), v(s + 1, 0), minv(s + 1);
    std::vector<int> match(s + 1, 0), way(s + 1, 0);  // match[col] = row
    std::vector<char> used(s + 1);
    for (int i = 1; i <= s; i++) {
        match[0] = i;
        int j0 = 0;
        std::fill(minv.begin(), minv.end(), INF);
        std::fill(used.begin(), used.end(), 0);
        do {
            used[j0] = 1;
            const int i0 = match[j0];
            int64_t delta = INF;
            int j1 = 0;
            for (int j = 1; j <= s; j++) {
                if (used[j]) continue;
                const int64_t cur = cost(i0 - 1, j - 1) - u[i0] - v[j];
                if (cur < minv[j]) {
                    minv[j] = cur;
                    way[j] = j0;
                }
                if (minv[j] < delta) {
                    delta = minv[j];
                    j1 = j;
                }
            }
            for (int j = 0; j <= s; j++) {
                if (used[j]) {
                    u[match[j]] += delta;
                    v[j] -= delta;
                } else {
                    minv[j] -= delta;
                }
            }
            j0 = j1;
        } while (match[j0] != 0);
        do {
            const int j1 = way[j0];
            match[j0] = match[j1];
            j0 = j1;
        } while (j0);
    }
    int64_t total = 0;
    for (int j = 1; j <= s; j++) {
        const int i = match[j];
        if (i >= 1 && i <= n && j <= m) total += w[(size_t)(i - 1) * m + (j - 1)];
    }
    return total;
}

int read_set(const ebic_bicluster *b, int32_t n, int32_t rows, int32_t cols,
             std::vector<Bic> *out) {
    if (n < 0 || (n > 0 && !b)) return fail(EBIC_ERR_INVALID_ARG, "bad bicluster list");
    out->resize(n);
    for (int32_t i = 0; i < n; i++) {
        const ebic_bicluster &x = b[i];
        if (x.n_rows < 0 || x.n_cols < 0 || (x.n_rows > 0 && !x.rows) ||
            (x.n_cols > 0 && !x.cols))
            return fail(EBIC_ERR_INVALID_ARG, "bicluster %d: bad row or column list", i);
        Bic &o = (*out)[i];
        o.rows.assign(x.rows, x.rows + x.n_rows);
        o.cols.assign(x.cols, x.cols + x.n_cols);
        for (int32_t r : o.rows)
            if (r < 0 || r >= rows) return fail(EBIC_ERR_INVALID_ARG, "bicluster %d: row %d", i, r);
        for (int32_t c : o.cols)
            if (c < 0 || c >= cols) return fail(EBIC_ERR_INVALID_ARG, "bicluster %d: col %d", i, c);
        std::sort(o.rows.begin(), o.rows.end());
        o.rows.erase(std::unique(o.rows.begin(), o.rows.end()), o.rows.end());
        std::sort(o.cols.begin(), o.cols.end());
        o.cols.erase(std::unique(o.cols.begin(), o.cols.end()), o.cols.end());
    }
    return EBIC_OK;
}

}  // namespace

int ce_score(const ebic_bicluster *found, int32_t n_found, const ebic_bicluster *truth,
             int32_t n_truth, int32_t rows, int32_t cols, double *score, double *ce) {
    if (!score || !ce) return fail(EBIC_ERR_INVALID_ARG, "NULL output");
    if (rows < 1 || cols < 1) return fail(EBIC_ERR_INVALID_ARG, "bad matrix shape");
    std::vector<Bic> f, t;
    int rc = read_set(found, n_found, rows, cols, &f);
    if (rc == EBIC_OK) rc = read_set(truth, n_truth, rows, cols, &t);
    if (rc) return rc;
    std::vector<int64_t> w((size_t)n_found * n_truth);
    for (int32_t i = 0; i < n_found; i++)
        for (int32_t j = 0; j < n_truth; j++)
            w[(size_t)i * n_truth + j] = shared(f[i].rows, t[j].rows) * shared(f[i].cols, t[j].cols);
    const int64_t d_max = max_assignment(w, n_found, n_truth);
    // |U|: per row, the union of the columns of every bicluster holding it
    std::vector<std::vector<int32_t>> by_row(rows);
    for (const std::vector<Bic> *set : {&f, &t})
        for (size_t q = 0; q < set->size(); q++)
            for (int32_t r : (*set)[q].rows) by_row[r].push_back((int32_t)(set == &f ? q : n_found + q));
    std::vector<char> mark(cols, 0);
    std::vector<int32_t> touched;
    int64_t u = 0;
    for (int32_t r = 0; r < rows; r++) {
        if (by_row[r].empty()) continue;
        for (int32_t id : by_row[r]) {
            const Bic &b = id < n_found ? f[id] : t[id - n_found];
            for (int32_t c : b.cols)
                if (!mark[c]) {
                    mark[c] = 1;
                    touched.push_back(c);
                }
        }
        u += (int64_t)touched.size();
        for (int32_t c : touched) mark[c] = 0;
        touched.clear();
    }
    if (u == 0) {  // no cells on either side: nothing to tell apart
        *score = 1.0;
        *ce = 0.0;
        return EBIC_OK;
    }
    *score = (double)d_max / (double)u;
    *ce = (double)(u - d_max) / (double)u;
    return EBIC_OK;
}

}  // namespace ebic
