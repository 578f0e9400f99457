// Autotuner inside the library (imq_tree_params.autotune): after the build,
// the fastest configuration of the tree whose error stays within a target
// (the same search as the Python tuner of the binding).
//
// The error of a configuration is measured, never modelled: the product of
// a fixed pseudo-random weight vector (uniform in [-1, 1)) is compared with
// exact FP64 direct sums on a fixed sample of rows (imq_rows_exact), by the
// relative 2-norm over those rows.  The cost model of Sec. 2.3 (eq.
// total_cost) is not evaluated; the time of a configuration is measured with
// HIP events on the caller's stream (the fastest of two batches of products
// after two untimed ones).  Search, for each internal precision (FP32, FP64):
//   1. the uniform translation order is lowered from p while the error stays
//      within 0.8 x target;
//   2. per level, deepest first, its order is lowered further while it does
//      (the lifted vertical offset c makes the deep levels, whose boxes are
//      small against c, converge fastest); then, since orders that fill the
//      same 16-row matrix-core tiles cost the same, each level is raised to
//      the top of its tile and levels are moved down by whole tiles, the
//      most translation work first, while the error allows (kept if the
//      product is measured faster);
//   3. the M2L kernel (register streaming, staged GEMM, and for FP32 the
//      BF16x3 streaming) and the staged GEMM's pipeline depth and row split
//      are timed, then the near field's workgroup count beside the tree
//      passes;
// and the faster precision that reaches the target is kept.  The tree is
// left configured (orders, kernels) and records the precision, its error
// and time (imq_get_tree_info: tuned_prec, tuned_err, tuned_ms).  Leaf
// capacity is a build parameter: comparing capacities means building one
// tree per capacity and comparing their tuned times.
#include "device.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

namespace imq {

namespace {

// 64-bit linear congruential generator (Knuth's MMIX constants), top 53 bits.
struct Lcg {
    uint64_t s;
    double uniform()
    {
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        return double(s >> 11) * (1.0 / 9007199254740992.0);
    }
};

struct Tuner {
    imq_tree t;
    hipStream_t s;
    int64_t N = 0;
    int nrows = 0;
    DevBuf u, b, rows, exact;
    std::vector<double> hb, hex;
    std::vector<int64_t> hrows;
    hipEvent_t e0 = nullptr, e1 = nullptr;

    ~Tuner()
    {
        dev_free(u);
        dev_free(b);
        dev_free(rows);
        dev_free(exact);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }

    imq_status setup(int64_t n)
    {
        N = n;
        nrows = int(std::min<int64_t>(1000, N));
        Lcg g{0x9e3779b97f4a7c15ull};
        std::vector<double> hu(static_cast<size_t>(N));
        for (auto &v : hu) v = 2.0 * g.uniform() - 1.0;
        // distinct rows drawn uniformly (repeats rejected), in increasing order
        std::vector<char> used(static_cast<size_t>(N), 0);
        while (int(hrows.size()) < nrows) {
            const int64_t r = std::min<int64_t>(N - 1, int64_t(g.uniform() * double(N)));
            if (!used[size_t(r)]) {
                used[size_t(r)] = 1;
                hrows.push_back(r);
            }
        }
        std::sort(hrows.begin(), hrows.end());
        IMQ_HIP(dev_alloc(u, sizeof(double) * size_t(N)));
        IMQ_HIP(dev_alloc(b, sizeof(double) * size_t(N)));
        IMQ_HIP(dev_alloc(rows, sizeof(int64_t) * size_t(nrows)));
        IMQ_HIP(dev_alloc(exact, sizeof(double) * size_t(nrows)));
        IMQ_HIP(hipMemcpy(u.p, hu.data(), sizeof(double) * hu.size(), hipMemcpyHostToDevice));
        IMQ_HIP(hipMemcpy(rows.p, hrows.data(), sizeof(int64_t) * hrows.size(), hipMemcpyHostToDevice));
        imq_status st = imq_rows_exact(t, 1, u.as<double>(), N, nrows, rows.as<int64_t>(), exact.as<double>(),
                                       nrows, s);
        if (st != IMQ_OK) return st;
        hex.resize(size_t(nrows));
        hb.resize(size_t(N));
        IMQ_HIP(hipMemcpyAsync(hex.data(), exact.p, sizeof(double) * hex.size(), hipMemcpyDeviceToHost, s));
        IMQ_HIP(hipStreamSynchronize(s));
        IMQ_HIP(hipEventCreate(&e0));
        IMQ_HIP(hipEventCreate(&e1));
        return IMQ_OK;
    }

    // relative 2-norm error of the current configuration on the sampled rows
    imq_status error(imq_prec prec, double &err)
    {
        imq_status st = imq_matvec(t, 1, IMQ_F64, u.p, N, b.p, N, prec, s);
        if (st != IMQ_OK) return st;
        IMQ_HIP(hipMemcpyAsync(hb.data(), b.p, sizeof(double) * hb.size(), hipMemcpyDeviceToHost, s));
        IMQ_HIP(hipStreamSynchronize(s));
        double num = 0.0, den = 0.0;
        for (int i = 0; i < nrows; ++i) {
            const double d = hb[size_t(hrows[size_t(i)])] - hex[size_t(i)];
            num += d * d;
            den += hex[size_t(i)] * hex[size_t(i)];
        }
        err = den > 0.0 ? std::sqrt(num / den) : std::sqrt(num);
        return IMQ_OK;
    }

    // ms per product: the fastest of two batches of five, after two untimed
    imq_status time(imq_prec prec, double &ms)
    {
        imq_status st;
        for (int i = 0; i < 2; ++i)
            if ((st = imq_matvec(t, 1, IMQ_F64, u.p, N, b.p, N, prec, s)) != IMQ_OK) return st;
        ms = 1e30;
        for (int batch = 0; batch < 2; ++batch) {
            IMQ_HIP(hipEventRecord(e0, s));
            for (int i = 0; i < 5; ++i)
                if ((st = imq_matvec(t, 1, IMQ_F64, u.p, N, b.p, N, prec, s)) != IMQ_OK) return st;
            IMQ_HIP(hipEventRecord(e1, s));
            IMQ_HIP(hipEventSynchronize(e1));
            float x = 0.0f;
            IMQ_HIP(hipEventElapsedTime(&x, e0, e1));
            ms = std::min(ms, double(x) / 5.0);
        }
        return IMQ_OK;
    }
};

}  // namespace

imq_status autotune_tree(imq_tree_s *t, double tol, hipStream_t s)
{
    const int nlev = t->h.nlev, p = t->h.p;
    if (nlev > IMQ_MAX_LEVELS + 1) { set_error("autotune: too many levels"); return IMQ_EINVAL; }
    std::vector<char> active(size_t(nlev), 0);      // levels with translations
    for (int l = 0; l < nlev; ++l)
        active[size_t(l)] = t->g_m2l.level_task_begin[size_t(l) + 1] > t->g_m2l.level_task_begin[size_t(l)];
    Tuner tu;
    tu.t = t;
    tu.s = s;
    imq_status st = tu.setup(t->h.N);
    if (st != IMQ_OK) return st;
    const double budget = 0.8 * tol;
    struct Best {
        bool ok = false;
        imq_prec prec = IMQ_PREC_FP64;
        std::vector<int> orders;
        imq_kernel_config kc{};
        double err = 0.0, ms = 1e30;
    } best;
    for (imq_prec prec : {IMQ_PREC_FP32, IMQ_PREC_FP64}) {
        std::vector<int> orders(size_t(nlev), p);
        imq_kernel_config kc{};
        if ((st = imq_set_kernel_config(t, &kc)) != IMQ_OK) return st;
        if ((st = imq_set_level_orders(t, nlev, orders.data())) != IMQ_OK) return st;
        double err;
        if ((st = tu.error(prec, err)) != IMQ_OK) return st;
        if (!(err <= budget)) continue;
        // 1. the uniform order
        while (orders[0] > 2) {
            std::vector<int> trial(orders);
            for (int &o : trial) --o;
            if ((st = imq_set_level_orders(t, nlev, trial.data())) != IMQ_OK) return st;
            double e;
            if ((st = tu.error(prec, e)) != IMQ_OK) return st;
            if (!(e <= budget)) break;
            orders = trial;
            err = e;
        }
        // 2. each level with translations, deepest first
        for (int l = nlev - 1; l >= 0; --l) {
            if (!active[size_t(l)]) continue;
            while (orders[size_t(l)] > 1) {
                std::vector<int> trial(orders);
                --trial[size_t(l)];
                if ((st = imq_set_level_orders(t, nlev, trial.data())) != IMQ_OK) return st;
                double e;
                if ((st = tu.error(prec, e)) != IMQ_OK) return st;
                if (!(e <= budget)) break;
                orders = trial;
                err = e;
            }
        }
        // 2b. orders that fill the same 16-row tiles of a translation cost the
        // same matrix-core work: every translated level to the top of its
        // tile (less error at no matrix-core cost), then levels down by whole
        // tiles, the ones with the most translation work first, within the
        // budget.  The shifts and L2P grow with the orders and levels of
        // different tile counts run as separate launches, so the result is
        // kept only if the product is measured faster than with the greedy
        // orders.
        {
            const std::vector<int> greedy(orders);
            const double greedy_err = err;
            const auto nrb = [](int o) { return ((o + 1) * (o + 2) / 2 + 15) / 16; };
            const auto top = [&](int o) {
                while (o + 1 <= p && nrb(o + 1) == nrb(o)) ++o;
                return o;
            };
            std::vector<int> raised(orders);
            for (int l = 0; l < nlev; ++l)
                if (active[size_t(l)]) raised[size_t(l)] = top(orders[size_t(l)]);
            if (raised != orders) {
                if ((st = imq_set_level_orders(t, nlev, raised.data())) != IMQ_OK) return st;
                double e;
                if ((st = tu.error(prec, e)) != IMQ_OK) return st;
                if (e <= budget) {
                    orders = raised;
                    err = e;
                }
            }
            std::vector<int> lv;
            for (int l = 0; l < nlev; ++l)
                if (active[size_t(l)]) lv.push_back(l);
            const HostTree &h = t->h;
            const auto work = [&](int l) {
                return double(h.v_off[h.level_begin[l + 1]] - h.v_off[h.level_begin[l]]) * nrb(orders[size_t(l)]);
            };
            std::stable_sort(lv.begin(), lv.end(), [&](int a, int b) { return work(a) > work(b); });
            for (int l : lv)
                while (nrb(orders[size_t(l)]) > 1) {
                    int lower = orders[size_t(l)];
                    while (lower > 1 && nrb(lower) == nrb(orders[size_t(l)])) --lower;
                    std::vector<int> trial(orders);
                    trial[size_t(l)] = lower;
                    if ((st = imq_set_level_orders(t, nlev, trial.data())) != IMQ_OK) return st;
                    double e;
                    if ((st = tu.error(prec, e)) != IMQ_OK) return st;
                    if (!(e <= budget)) break;
                    orders = trial;
                    err = e;
                }
            if (orders != greedy) {
                double tg, tr;
                if ((st = imq_set_level_orders(t, nlev, greedy.data())) != IMQ_OK) return st;
                if ((st = tu.time(prec, tg)) != IMQ_OK) return st;
                if ((st = imq_set_level_orders(t, nlev, orders.data())) != IMQ_OK) return st;
                if ((st = tu.time(prec, tr)) != IMQ_OK) return st;
                if (!(tr < tg)) {
                    orders = greedy;
                    err = greedy_err;
                }
            }
        }
        if ((st = imq_set_level_orders(t, nlev, orders.data())) != IMQ_OK) return st;
        // 3. kernels and launch shapes
        imq_kernel_config bk{};
        double bms = 1e30;
        const bool wide = *std::max_element(orders.begin(), orders.end()) >= 12;   // above 80 coefficients
        for (int mode : {0, 1, 2, 3}) {
            if (prec == IMQ_PREC_FP64 && mode == 2) continue;      // the BF16 parts serve FP32 only
            if (mode == 3 && !wide) continue;                      // the same kernels as mode 0
            for (int kcv : {16, 32, 64}) {
                if (prec == IMQ_PREC_FP64 && kcv > 32) continue;
                if (mode == 3 && kcv != 16) continue;              // mode 3 has no staged GEMM
                for (int sp : {1, 2}) {
                    if (mode == 3 && sp != 1) continue;
                    imq_kernel_config c{};
                    c.m2l_mode = mode;
                    c.m2l_kc = kcv;
                    c.m2l_split = sp;
                    if ((st = imq_set_kernel_config(t, &c)) != IMQ_OK) return st;
                    double ms;
                    if ((st = tu.time(prec, ms)) != IMQ_OK) return st;
                    if (ms < bms) { bms = ms; bk = c; }
                }
            }
        }
        const imq_kernel_config shape = bk;
        for (int wg : {2048, 2560, 3072, 3584}) {
            imq_kernel_config c = shape;
            c.p2p_wg = wg;
            if ((st = imq_set_kernel_config(t, &c)) != IMQ_OK) return st;
            double ms;
            if ((st = tu.time(prec, ms)) != IMQ_OK) return st;
            if (ms < bms) { bms = ms; bk = c; }
        }
        if (!best.ok || bms < best.ms) {
            best.ok = true;
            best.prec = prec;
            best.orders = orders;
            best.kc = bk;
            best.err = err;
            best.ms = bms;
        }
    }
    if (!best.ok) {
        set_error("autotune: no precision reaches the target error at order p; build with a larger order_p");
        return IMQ_EINVAL;
    }
    if ((st = imq_set_level_orders(t, nlev, best.orders.data())) != IMQ_OK) return st;
    if ((st = imq_set_kernel_config(t, &best.kc)) != IMQ_OK) return st;
    double err;
    if ((st = tu.error(best.prec, err)) != IMQ_OK) return st;
    t->tuned_prec = int(best.prec);
    t->tuned_err = err;
    t->tuned_ms = best.ms;
    return IMQ_OK;
}

}  // namespace imq
