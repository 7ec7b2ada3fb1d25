// tables.cpp -- host construction of the device-resident tables:
// Sobol direction numbers, the per-wave lane table, bridge plans and
// principal-component factors.  Everything here is computed once per process
// (direction numbers, plans) or once per distinct (n, dt) (PCA factors).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <utility>
#include <vector>

#include "qcpw_host.h"

namespace qcpw {

#include "joe_kuo_data.inc"

// Direction numbers as 32-bit binary fractions v_i = m_i / 2^i (Sec. 2.2.2).
// Dividing eqn:SobolRecurrenceRelation by 2^i gives the recurrence on the
// fractions themselves:  v_i = c_1 v_{i-1} ^ ... ^ c_{q-1} v_{i-q+1}
//                              ^ v_{i-q} ^ (v_{i-q} >> q).
// Dimension 0 (polynomial 1, degree 0) has v_i = 2^-i: the identity matrix.
void build_direction_numbers(std::vector<uint32_t> &dir)
{
    dir.assign((size_t)QCPW_TAB_DIMS * 32, 0u);
    for (int j = 0; j < QCPW_TAB_DIMS; ++j) {
        uint32_t *v = &dir[(size_t)j * 32];
        const uint32_t poly = qcpw_jk_poly[j];
        int q = 31 - __builtin_clz(poly);   // degree
        if (q == 0) {
            for (int i = 0; i < 32; ++i) v[i] = 1u << (31 - i);
            continue;
        }
        for (int i = 0; i < q && i < 32; ++i) v[i] = qcpw_jk_minit[j][i] << (31 - i);
        for (int i = q; i < 32; ++i) {
            uint32_t x = v[i - q] ^ (v[i - q] >> q);
            for (int k = 1; k < q; ++k)
                if ((poly >> (q - k)) & 1u) x ^= v[i - k];
            v[i] = x;
        }
    }
}

// lane[j][t] = XOR_{b : bit b of gray(t)} dir[j][b], t = 0..63.
void build_lane_table(const std::vector<uint32_t> &dir, std::vector<uint32_t> &lane)
{
    lane.assign((size_t)QCPW_TAB_DIMS * 64, 0u);
    for (int j = 0; j < QCPW_TAB_DIMS; ++j)
        for (int t = 0; t < 64; ++t) {
            uint32_t g = (uint32_t)(t ^ (t >> 1)), y = 0;
            for (int b = 0; g; ++b, g >>= 1)
                if (g & 1u) y ^= dir[(size_t)j * 32 + b];
            lane[(size_t)j * 64 + t] = y;
        }
}

// Bridge plan for n grid points (Sec. 4.4 for any n).  The normals are
// assigned in breadth-first order: the terminal point W(n dt) takes
// dimension 1, then every interval (l, r) with r - l >= 2, taken from a FIFO
// that starts with (0, n), takes the next dimension for its midpoint
// m = floor((l + r) / 2) and queues (l, m) and (m, r).  The kernel walks
// the same intervals depth first (left child before right child), which
// needs only a stack of right end points; `pops` records, before each
// midpoint, how many finished leaves return control to a pending right
// subtree.  Returns the maximum stack depth.
int build_bridge_plan(int n, std::vector<PlanStep> &steps, std::vector<PlanStep64> &steps64)
{
    steps.clear();
    steps64.clear();
    if (n <= 0) return 0;
    std::map<std::pair<int, int>, int> dim_of;
    {
        std::deque<std::pair<int, int>> fifo;
        fifo.emplace_back(0, n);
        int next_dim = 2;
        while (!fifo.empty()) {
            auto iv = fifo.front();
            fifo.pop_front();
            if (iv.second - iv.first < 2) continue;
            int m = (iv.first + iv.second) / 2;
            dim_of[iv] = next_dim++;
            fifo.emplace_back(iv.first, m);
            fifo.emplace_back(m, iv.second);
        }
    }
    int sp = 0, max_sp = 0;   // stack depth as the kernel sees it
    auto add = [&](int dim, int m, int pops, double wl, double wr, double sd) {
        PlanStep s;
        s.lds_off = qcpw_row_word(dim - 1);
        if (steps.empty()) {
            s.slot = 0;                 // terminal point: no stack access
        } else if (pops == 0) {
            s.slot = sp++;              // push R
        } else {
            s.slot = sp - pops;         // R = stack[slot], L = stack[slot + 1] if pops >= 2
            sp = s.slot + 1;
        }
        max_sp = std::max(max_sp, sp);
        s.pops = pops;
        s.dim = dim;
        s.wl = (float)wl;
        s.wr = (float)wr;
        s.sd = (float)sd;
        s.mf = (float)m;
        steps.push_back(s);
        steps64.push_back(PlanStep64{wl, wr, sd, (double)m});
    };
    add(1, n, 0, 0.0, 0.0, qcpw_csqrt((double)n));   // terminal point
    bool consistent = true;   // the compile-time bridges walk the same intervals

    int pending = 0, depth = 0, max_depth = 0;
    // iterative depth-first walk: frame = (l, r, state)
    struct Frame { int l, r, state; };
    std::vector<Frame> st;
    st.push_back({0, n, 0});
    while (!st.empty()) {
        Frame &f = st.back();
        if (f.r - f.l < 2) {             // leaf: "L = R" (paired with the next pop)
            st.pop_back();
            continue;
        }
        int m = (f.l + f.r) / 2;
        if (f.state == 0) {
            double len = f.r - f.l;
            if (n <= QCPW_FIXED_MAX_N &&
                (qcpw_bridge_dim(n, f.l, f.r) != dim_of[{f.l, f.r}] ||
                 qcpw_bridge_step(n, f.l, f.r) != (int)steps.size()))
                consistent = false;
            add(dim_of[{f.l, f.r}], m, pending, (f.r - m) / len, (m - f.l) / len,
                qcpw_csqrt((double)(m - f.l) * (double)(f.r - m) / len));
            pending = 0;
            ++depth;
            if (depth > max_depth) max_depth = depth;
            f.state = 1;
            st.push_back({f.l, m, 0});
        } else if (f.state == 1) {       // left subtree done: R = pop()
            ++pending;
            --depth;
            f.state = 2;
            st.push_back({m, f.r, 0});
        } else {
            st.pop_back();
        }
    }
    if (!consistent) return -1;
    return std::max(max_depth, max_sp);
}

// Principal components of Sigma_{kl} = dt min(k, l), k, l = 1..n, in closed
// form: eigenvalues dt / (4 sin^2((2i-1) pi / (2(2n+1)))), eigenvectors
// sqrt(2/(n+1/2)) sin((2i-1) k pi / (2n+1)), i = 1..n (largest first, first
// entry positive).  A_{k,i} = sqrt(lambda_i) v_i(k), row-major.  The angle is
// reduced exactly in integers before it is scaled by pi.
void build_pca_factor(int n, double dt, std::vector<double> &A)
{
    A.assign((size_t)n * n, 0.0);
    const long period = 2L * (2 * n + 1);
    const double norm = std::sqrt(2.0 / (n + 0.5));
    for (int i = 1; i <= n; ++i) {
        double half = std::sin(M_PI * (2 * i - 1) / (double)period);
        double root_lambda = std::sqrt(dt) / (2.0 * half);
        for (int k = 1; k <= n; ++k) {
            long a = ((long)(2 * i - 1) * (long)k) % period;
            A[(size_t)(k - 1) * n + (i - 1)] = root_lambda * norm * std::sin(M_PI * (double)a / (2 * n + 1));
        }
    }
}

void build_factor(int path, int n, double dt, std::vector<double> &A)
{
    A.assign((size_t)n * n, 0.0);
    if (n <= 0) return;
    if (path == QCPW_PATH_PCA) {
        build_pca_factor(n, dt, A);
        return;
    }
    if (path == QCPW_PATH_STANDARD) {
        for (int k = 0; k < n; ++k)
            for (int i = 0; i <= k; ++i) A[(size_t)k * n + i] = std::sqrt(dt);
        return;
    }
    // bridge: apply the plan to every unit vector (column by column), with
    // the stack slots exactly as the kernels use them
    std::vector<PlanStep> steps;
    std::vector<PlanStep64> s64;
    const int depth = build_bridge_plan(n, steps, s64);
    if (depth < 0) {
        std::fill(A.begin(), A.end(), std::nan(""));   // plan self-check failed
        return;
    }
    std::vector<double> W(n + 1);
    for (int col = 0; col < n; ++col) {
        std::vector<double> stack(depth + 1, std::nan(""));
        double L = 0.0, R = 0.0;
        for (size_t s = 0; s < steps.size(); ++s) {
            double z = (steps[s].dim - 1 == col) ? std::sqrt(dt) : 0.0;
            if (s == 0) {
                R = s64[0].sd * z;
                W[n] = R;
                continue;
            }
            const int slot = steps[s].slot, pops = steps[s].pops;
            if (slot < 0 || slot >= depth || (pops >= 2 && slot + 1 >= depth)) {
                std::fill(A.begin(), A.end(), std::nan(""));   // a broken plan fails every check
                return;
            }
            if (pops == 0) {
                stack[slot] = R;
            } else {
                const double r = stack[slot];
                L = pops == 1 ? R : stack[slot + 1];
                R = r;
            }
            double Wm = s64[s].wl * L + s64[s].wr * R + s64[s].sd * z;
            R = Wm;
            W[(int)steps[s].mf] = Wm;
        }
        for (int k = 0; k < n; ++k) A[(size_t)k * n + col] = W[k + 1];
    }
}

}  // namespace qcpw
