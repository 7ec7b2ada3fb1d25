// tables.cpp -- host construction of the device-resident tables:
// Sobol direction numbers, the per-wave lane table, bridge plans and
// principal-component factors.  Everything here is computed once per process
// (direction numbers, plans) or once per distinct (n, dt) (PCA factors).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <deque>
#include <functional>
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

// Breadth-first dimensions of the bridge's intervals (as build_bridge_plan).
static std::map<std::pair<int, int>, int> bridge_dims(int n)
{
    std::map<std::pair<int, int>, int> dim_of;
    std::deque<std::pair<int, int>> fifo;
    fifo.emplace_back(0, n);
    int next_dim = 2;
    while (!fifo.empty()) {
        auto iv = fifo.front();
        fifo.pop_front();
        if (iv.second - iv.first < 2) continue;
        const int m = (iv.first + iv.second) / 2;
        dim_of[iv] = next_dim++;
        fifo.emplace_back(iv.first, m);
        fifo.emplace_back(m, iv.second);
    }
    return dim_of;
}

static uint32_t fbits(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

// Split-bridge plan for n (see qcpw_internal.h): events in depth-first
// order -- the terminal point, then top midpoints and subtrees -- and the
// Sobol dimension of every wave-uniform slot.  Slots: the terminal point and
// the top nodes take 0 .. 2^k - 1 in event order; each subtree then takes
// the next len - 1 slots, moved to the start of the next register when they
// would straddle one.  The terminal event's word 8 holds the event count.
// Returns the slots used, or 0 when n has no split plan.
int build_split_plan(int n, std::vector<uint32_t> &ev, std::vector<uint16_t> &slot_dim)
{
    ev.assign((size_t)QCPW_SPLIT_EVENTS * QCPW_EV_WORDS, 0u);
    slot_dim.assign(QCPW_SPLIT_SLOTS, 0);
    if (n < QCPW_SUB_MIN_LEN || n > QCPW_MAX_N) return 0;
    const int k = qcpw_split_level(n);
    const auto dim_of = bridge_dims(n);
    int e = 0, top_slot = 0, sub_slot = 1 << k;
    bool ok = true;
    auto head = [&](int kind, int len, int slot, int m) -> uint32_t * {
        uint32_t *w = &ev[(size_t)e * QCPW_EV_WORDS];
        w[0] = qcpw_ev_header(kind, len, slot / 64, slot % 64);
        w[1] = (uint32_t)m;
        w[2] = fbits((float)m);
        w[3] = fbits(8388608.0f + (float)m);
        ++e;
        return w;
    };
    {   // terminal point, dimension 1
        const int slot = top_slot++;
        uint32_t *w = head(QCPW_EV_TERMINAL, 0, slot, n);
        w[4] = (uint32_t)qcpw_row_word(0);
        w[7] = fbits((float)qcpw_csqrt((double)n));
        slot_dim[slot] = 1;
    }
    std::function<void(int, int, int)> visit = [&](int l, int r, int level) {
        if (!ok) return;
        const int len = r - l;
        if (level == k) {
            if (len < QCPW_SUB_MIN_LEN || len > QCPW_SUB_MAX_LEN) { ok = false; return; }
            const int nodes = len - 1;
            if (sub_slot / 64 != (sub_slot + nodes - 1) / 64) sub_slot = (sub_slot / 64 + 1) * 64;
            if (sub_slot + nodes > QCPW_SPLIT_SLOTS) { ok = false; return; }
            uint32_t *w = head(QCPW_EV_SUB, len, sub_slot, l);
            // the subtree's midpoints in depth-first order; per level the
            // first node's row, the others following it one row apart (in
            // the upper region when the level's rows cross the gap)
            int t = 0;
            int first[QCPW_SUB_LEVELS], last[QCPW_SUB_LEVELS];
            for (int j = 0; j < QCPW_SUB_LEVELS; ++j) first[j] = last[j] = -1;
            std::function<void(int, int)> walk = [&](int lo, int hi) {
                if (hi - lo < 2) return;
                const int m = (lo + hi) / 2;
                auto it = dim_of.find({l + lo, l + hi});
                if (it == dim_of.end() || qcpw_sub_step(len, lo, hi) != t) { ok = false; return; }
                const QcpwSubPos p = qcpw_sub_pos(len, t);
                const int row = it->second - 1;
                if (p.level >= QCPW_SUB_LEVELS || (p.index == 0) != (first[p.level] < 0) ||
                    (p.index > 0 && row != first[p.level] + p.index)) { ok = false; return; }
                if (p.index == 0) first[p.level] = row;
                last[p.level] = row;
                slot_dim[sub_slot + t] = (uint16_t)it->second;
                ++t;
                walk(lo, m);
                walk(m, hi);
            };
            walk(0, len);
            if (t != nodes) ok = false;
            for (int j = 0; ok && j < QCPW_SUB_LEVELS && first[j] >= 0; ++j) {
                if (last[j] < QCPW_LDS_GAP_ROWS) w[4 + j] = (uint32_t)qcpw_row_word(first[j]);
                else if (first[j] >= QCPW_LDS_GAP_ROWS - QCPW_LDS_DUP_ROWS) w[4 + j] = (uint32_t)qcpw_row_word_hi(first[j]);
                else ok = false;
            }
            sub_slot += nodes;
            return;
        }
        const int m = (l + r) / 2;
        auto it = dim_of.find({l, r});
        if (it == dim_of.end()) { ok = false; return; }
        const int slot = top_slot++;
        uint32_t *w = head(QCPW_EV_TOP, 0, slot, m);
        w[4] = (uint32_t)qcpw_row_word(it->second - 1);
        w[5] = fbits((float)((double)(r - m) / len));
        w[6] = fbits((float)((double)(m - l) / len));
        w[7] = fbits((float)qcpw_csqrt((double)(m - l) * (double)(r - m) / len));
        w[8] = (uint32_t)l;
        w[9] = (uint32_t)r;
        slot_dim[slot] = (uint16_t)it->second;
        visit(l, m, level + 1);
        visit(m, r, level + 1);
    };
    visit(0, n, 0);
    // the kernel reads the terminal point's and the top nodes' parts from register 0
    if (!ok || e != (2 << k) || e > QCPW_SPLIT_EVENTS || top_slot > 64) return 0;
    ev[8] = (uint32_t)e;
    return sub_slot;
}

// The factor A (n x n, row-major) that the split plan's walk applies, in
// FP64 (the kernel's steps with FP64 weights): for every unit vector z the
// events and subtrees are walked exactly as the FP32 kernel walks them.
void split_plan_factor(int n, double dt, const std::vector<uint32_t> &ev, std::vector<double> &A)
{
    A.assign((size_t)n * n, std::nan(""));
    const int n_ev = (int)ev[8];
    auto word_dim = [](uint32_t w) { return qcpw_word_row(w) + 1; };
    const double sdt = std::sqrt(dt);
    for (int col = 0; col < n; ++col) {
        std::vector<double> W(n + 1, std::nan(""));
        W[0] = 0.0;
        auto zof = [&](int dim) { return dim - 1 == col ? sdt : 0.0; };
        const uint32_t *t = ev.data();
        double R = (double)qcpw_csqrt((double)n) * zof(word_dim(t[4])), L = 0.0;
        W[n] = R;
        std::vector<double> stack;
        for (int e = 1; e < n_ev; ++e) {
            const uint32_t *w = ev.data() + (size_t)e * QCPW_EV_WORDS;
            const int kind = w[0] & 255, len = (w[0] >> 8) & 255, m = (int)w[1];
            if (kind == QCPW_EV_TOP) {
                // FP64 weights of the interval (l, r) the event names
                const int l = (int)w[8], r = (int)w[9];
                const double len_d = r - l;
                const double M = (r - m) / len_d * L + (m - l) / len_d * R +
                                 qcpw_csqrt((double)(m - l) * (double)(r - m) / len_d) * zof(word_dim(w[4]));
                W[m] = M;
                stack.push_back(R);
                R = M;
            } else {
                int t_node = 0;
                std::function<void(int, int, double, double)> walk = [&](int lo, int hi, double WL, double WR) {
                    if (hi - lo < 2) return;
                    const int mm = (lo + hi) / 2;
                    const double wl = (double)(hi - mm) / (double)(hi - lo), wr = (double)(mm - lo) / (double)(hi - lo);
                    const double sd = qcpw_csqrt((double)(mm - lo) * (double)(hi - mm) / (double)(hi - lo));
                    const QcpwSubPos p = qcpw_sub_pos(len, t_node);
                    const uint32_t off = w[4 + p.level] + 64u * (uint32_t)p.index;
                    ++t_node;
                    const double Y = wl * WL + wr * WR + sd * zof(word_dim(off));
                    W[m + mm] = Y;
                    walk(lo, mm, WL, Y);
                    walk(mm, hi, Y, WR);
                };
                walk(0, len, L, R);
                L = R;
                if (!stack.empty()) {
                    R = stack.back();
                    stack.pop_back();
                }
            }
        }
        for (int kk = 0; kk < n; ++kk) A[(size_t)kk * n + col] = W[kk + 1];
    }
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
