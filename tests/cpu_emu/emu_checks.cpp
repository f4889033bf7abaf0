// Checks of the HIP library run on the CPU under the emulation in
// emu_rt.cpp, built with AddressSanitizer and UndefinedBehaviorSanitizer:
//   batch K MODE   nine contexts stepped alone and then together through
//                  pf_batch_run (MODE 0), its graph mode (1; 3: in runs of 10
//                  iterations, one graph replayed) or pf_batch_run_noalloc
//                  (2); results compared bit for bit
//   traj           pf_run_traj's rows against pf_estimate after each step
//   stream         k_step_flex against k_step on PEs both can run (one PE
//                  per workgroup with the log-weights in HBM, and several PEs
//                  per workgroup through pes_per_wg), every traced output
//                  compared after each iteration; then contexts of up to
//                  65536 particles per PE through pf_step, their ancestors
//                  checked against systematic resampling of the traced weights
//   master         k_master against master_block, bit for bit
#include "src/arna.hip"
#include <algorithm>
#include <random>
#include <vector>

// (the multi-iteration kernel is not built here: its cooperative launch
// needs every workgroup resident at once)
void *arna_run_kernel(uint32_t, uint32_t, uint32_t) { return nullptr; }
extern "C" void emu_set_fill(int v);
// CPU emulation of the batched-run test: nine contexts stepped alone and then
// together (pf_batch_run), results compared bit for bit; ASan watches every
// device buffer and the LDS block of every workgroup.

struct Case {
    uint32_t F, M, np, W, H, mode, lik, patch, block, groups;
    float fixed, bg, noise;
    uint64_t seed;
    uint32_t ppw = 0;   // PEs per workgroup
};

static pf_config make_cfg(const Case &c) {
    pf_config p;
    memset(&p, 0, sizeof(p));
    p.struct_size = sizeof(pf_config);
    p.n_filters = c.F; p.n_pe = c.M; p.n_per_pe = c.np; p.width = c.W; p.height = c.H;
    p.patch = c.patch; p.mode = c.mode; p.init_mode = 0; p.lik_mode = c.lik;
    p.fixed_ratio = c.fixed; p.initial_ratio = 0.1f; p.eff_cutoff = 0.99f; p.psf_sigma = 1.5f;
    p.background = c.bg; p.noise_sigma = c.noise; p.q = 0.5f; p.sigma_I = 0.5f;
    p.debug = 0; p.ring_groups = c.groups; p.block_size = c.block; p.launch = 0; p.seed = c.seed;
    p.pes_per_wg = c.ppw;
    p.stream = nullptr;
    return p;
}

struct Inputs { std::vector<float> truth, frames; uint64_t stride; };

static Inputs make_inputs(const Case &c, int K, std::mt19937_64 &rng) {
    Inputs in;
    std::uniform_real_distribution<double> U(0, 1);
    std::normal_distribution<double> Nd(0, 1);
    in.truth.assign(5 * c.F, 0.f);
    for (uint32_t f = 0; f < c.F; ++f) {
        in.truth[5 * f + 0] = 20 + U(rng) * (c.W - 40);
        in.truth[5 * f + 1] = 20 + U(rng) * (c.H - 40);
        in.truth[5 * f + 2] = U(rng) - 0.5;
        in.truth[5 * f + 3] = U(rng) - 0.5;
        in.truth[5 * f + 4] = 12.f;
    }
    if (c.lik == PF_LIK_POINT) {
        in.stride = 2 * c.F;
        for (int k = 0; k < K; ++k)
            for (uint32_t f = 0; f < c.F; ++f) {
                in.frames.push_back(in.truth[5 * f] + (k + 1) * in.truth[5 * f + 2] + Nd(rng));
                in.frames.push_back(in.truth[5 * f + 1] + (k + 1) * in.truth[5 * f + 3] + Nd(rng));
            }
        return in;
    }
    in.stride = (uint64_t)c.W * c.H;
    for (int k = 0; k < K; ++k) {
        for (uint32_t y = 0; y < c.H; ++y)
            for (uint32_t x = 0; x < c.W; ++x) {
                double mu = c.bg;
                for (uint32_t f = 0; f < c.F; ++f) {
                    const double px = in.truth[5 * f] + (k + 1) * in.truth[5 * f + 2];
                    const double py = in.truth[5 * f + 1] + (k + 1) * in.truth[5 * f + 3];
                    mu += 12.0 * exp(-((x - px) * (x - px) + (y - py) * (y - py)) / (2 * 1.5 * 1.5));
                }
                double z;
                if (c.lik == PF_LIK_POISSON) {
                    std::poisson_distribution<int> P(mu);
                    z = P(rng);
                } else {
                    z = mu + c.noise * Nd(rng);
                }
                in.frames.push_back((float)z);
            }
    }
    return in;
}

struct Result { std::vector<float> st; std::vector<unsigned char> rec; std::vector<double> xg, lg, pe; std::vector<uint32_t> nex, nexn; uint64_t step; };

static void check(int rc, const char *w) {
    if (rc != PF_OK) { fprintf(stderr, "%s: %s (%d)\n", w, pf_strerror(rc), rc); exit(1); }
}

static Result grab(pf_ctx *c, const Case &cs) {
    Result r;
    r.st.resize(pf_debug_size(c, PF_DBG_STATE) / 4);
    check(pf_debug_get(c, PF_DBG_STATE, r.st.data(), r.st.size() * 4), "state");
    r.rec.resize(pf_debug_size(c, PF_DBG_PE_RECORDS));
    check(pf_debug_get(c, PF_DBG_PE_RECORDS, r.rec.data(), r.rec.size()), "rec");
    r.xg.resize(5 * cs.F); r.lg.resize(cs.F); r.pe.resize(cs.F); r.nex.resize(cs.F); r.nexn.resize(cs.F);
    pf_estimate_t e;
    memset(&e, 0, sizeof(e));
    e.x_global = r.xg.data(); e.log_mass_glob = r.lg.data(); e.pe_eff = r.pe.data();
    e.n_ex = r.nex.data(); e.n_ex_next = r.nexn.data();
    check(pf_estimate(c, &e), "estimate");
    r.step = e.step;
    return r;
}

static int batch_main(int K, int graph) {
    const int split = K > 40 ? 40 : K / 2;
    std::vector<Case> cases = {
        {1, 4, 256, 128, 128, 0, 0, 9, 0, 0, 0.1f, 5.f, 2.f, 1},
        {1, 4, 256, 128, 128, 1, 0, 9, 0, 0, 0.1f, 5.f, 2.f, 2},
        {2, 8, 300, 96, 80, 1, 0, 9, 0, 0, 0.1f, 5.f, 2.f, 3},
        {1, 6, 2500, 128, 128, 1, 0, 9, 0, 0, 0.1f, 5.f, 2.f, 4},
        {1, 4, 1000, 64, 48, 1, 2, 9, 0, 0, 0.1f, 10.f, 2.f, 5},
        {3, 5, 77, 128, 128, 0, 1, 9, 0, 0, 0.5f, 5.f, 1.f, 6},
        {1, 3, 200, 64, 64, 1, 0, 7, 0, 0, 0.1f, 5.f, 2.f, 7},
        {1, 5, 1000, 96, 80, 1, 0, 9, 512, 0, 0.1f, 5.f, 2.f, 8},
        {2, 8, 100, 96, 80, 1, 0, 9, 0, 4, 0.1f, 5.f, 2.f, 9},
        // several PEs per workgroup (batched k_step_flex), split PEs (batched
        // split launches)
        {1, 4, 256, 128, 128, 1, 0, 9, 0, 0, 0.1f, 5.f, 2.f, 10, 2},
        {2, 3, 130, 96, 80, 0, 1, 9, 0, 0, 0.5f, 5.f, 1.f, 11, 3},
        {1, 2, 5000, 96, 96, 1, 0, 9, 0, 0, 0.1f, 5.f, 2.f, 12},
        {1, 2, 4500, 64, 64, 1, 2, 9, 0, 0, 0.1f, 10.f, 2.f, 13},
    };
    if (getenv("EMU_CASES")) {   // case indices as digits and letters (a = 10), e.g. "013b"
        std::vector<Case> sel;
        for (const char *p = getenv("EMU_CASES"); *p; ++p)
            sel.push_back(cases[*p >= 'a' ? *p - 'a' + 10 : *p - '0']);
        cases = sel;
    }
    std::mt19937_64 rng(2024);
    std::vector<Inputs> ins;
    for (auto &c : cases) ins.push_back(make_inputs(c, K, rng));
    // device copies of the frames (plain host memory under the emulation)
    std::vector<float *> dfr;
    for (auto &in : ins) {
        float *d;
        hipMalloc(&d, in.frames.size() * 4);
        memcpy(d, in.frames.data(), in.frames.size() * 4);
        dfr.push_back(d);
    }
    std::vector<Result> solo;
    for (size_t i = 0; i < cases.size(); ++i) {
        pf_config cfg = make_cfg(cases[i]);
        pf_ctx *c;
        check(pf_init(&cfg, ins[i].truth.data(), &c), "init");
        check(pf_run(c, dfr[i], split, ins[i].stride), "run a");
        check(pf_run(c, dfr[i] + split * ins[i].stride, K - split, ins[i].stride), "run b");
        solo.push_back(grab(c, cases[i]));
        pf_destroy(c);
        fprintf(stderr, "solo case %zu done\n", i);
    }
    std::vector<pf_ctx *> ctx(cases.size());
    for (size_t i = 0; i < cases.size(); ++i) {
        pf_config cfg = make_cfg(cases[i]);
        check(pf_init(&cfg, ins[i].truth.data(), &ctx[i]), "init b");
    }
    pf_batch *b;
    check(pf_batch_create(ctx.data(), (uint32_t)ctx.size(), &b), "batch create");
    std::vector<const float *> p0, p1;
    std::vector<uint64_t> strides;
    for (size_t i = 0; i < cases.size(); ++i) {
        p0.push_back(dfr[i]);
        p1.push_back(dfr[i] + split * ins[i].stride);
        strides.push_back(ins[i].stride);
    }
    if (graph == 3) {   // graph mode in equal runs: one capture, replayed
        for (int t0 = 0; t0 < K; t0 += 10) {
            std::vector<const float *> pt;
            for (size_t i = 0; i < cases.size(); ++i) pt.push_back(dfr[i] + t0 * ins[i].stride);
            check(pf_batch_run(b, pt.data(), strides.data(), K - t0 < 10 ? K - t0 : 10, 1), "graph run");
        }
    } else if (graph == 2) {   // the entry point that allocates nothing
        const int big = pf_batch_run_noalloc(b, p0.data(), strides.data(), 100000);
        fprintf(stderr, "oversized no-alloc run: %d\n", big);
        if (big != PF_EUNSUPPORTED) return 3;
        check(pf_batch_run_noalloc(b, p0.data(), strides.data(), split), "noalloc a");
        check(pf_batch_run_noalloc(b, p1.data(), strides.data(), K - split), "noalloc b");
    } else {
        check(pf_batch_run(b, p0.data(), strides.data(), split, graph), "batch a");
        check(pf_batch_run(b, p1.data(), strides.data(), K - split, graph), "batch b");
    }
    int bad = 0;
    for (size_t i = 0; i < cases.size(); ++i) {
        Result r = grab(ctx[i], cases[i]);
        const Result &s = solo[i];
        const bool eq = r.st == s.st && r.rec == s.rec && r.xg == s.xg && r.lg == s.lg &&
                        r.pe == s.pe && r.nex == s.nex && r.nexn == s.nexn && r.step == s.step;
        size_t nd = 0;
        for (size_t j = 0; j < r.st.size(); ++j) nd += memcmp(&r.st[j], &s.st[j], 4) != 0;
        fprintf(stderr, "case %zu: batch %s solo (state values differing: %zu of %zu), step %llu\n", i,
                eq ? "==" : "!=", nd, r.st.size(), (unsigned long long)r.step);
        bad += !eq;
    }
    pf_batch_destroy(b);
    for (auto c : ctx) pf_destroy(c);
    for (auto d : dfr) hipFree(d);
    fprintf(stderr, bad ? "MISMATCH\n" : "ALL EQUAL\n");
    return bad ? 2 : 0;
}

// pf_run_traj in two calls against a stepwise run with pf_estimate after
// every iteration: the rows must be those estimates, bit for bit.
static int traj_main() {
    int bad = 0;
    const Case cases[] = {
        {2, 8, 300, 96, 80, 1, 0, 9, 0, 0, 0.1f, 5.f, 2.f, 3},
        {1, 4, 256, 128, 128, 0, 0, 9, 0, 0, 0.1f, 5.f, 2.f, 1},
        {1, 300, 64, 64, 64, 1, 0, 9, 0, 0, 0.1f, 5.f, 2.f, 11},    // more than 256 PEs
        {3, 5, 77, 128, 128, 1, 1, 9, 0, 0, 0.5f, 5.f, 1.f, 6},
        {1, 2, 5000, 96, 96, 1, 0, 9, 0, 0, 0.1f, 5.f, 2.f, 8},     // split PEs
        {1, 520, 16, 64, 64, 1, 0, 9, 0, 0, 0.1f, 5.f, 2.f, 9},     // master records
        {1, 530, 16, 64, 64, 1, 0, 9, 0, 0, 0.1f, 5.f, 2.f, 10, 4}, // and k_step_flex
    };
    std::mt19937_64 rng(7);
    for (const Case &cs : cases) {
        const int K = 9;
        Inputs in = make_inputs(cs, K, rng);
        float *d;
        hipMalloc(&d, in.frames.size() * 4);
        memcpy(d, in.frames.data(), in.frames.size() * 4);
        pf_config cfg = make_cfg(cs);
        pf_ctx *a, *b;
        check(pf_init(&cfg, in.truth.data(), &a), "init a");
        check(pf_init(&cfg, in.truth.data(), &b), "init b");
        pf_master_t *traj;
        hipMalloc(&traj, sizeof(pf_master_t) * K * cs.F);
        check(pf_run_traj(a, d, 4, in.stride, traj), "traj a");
        check(pf_run_traj(a, d + 4 * in.stride, K - 4, in.stride, traj + 4 * cs.F), "traj b");
        for (int k = 0; k < K; ++k) {
            check(pf_step(b, d + k * in.stride), "step");
            std::vector<double> xg(5 * cs.F), lg(cs.F), pe(cs.F), lz(cs.F);
            std::vector<uint32_t> nx(cs.F), nn(cs.F);
            pf_estimate_t e;
            memset(&e, 0, sizeof(e));
            e.x_global = xg.data(); e.log_mass_glob = lg.data(); e.pe_eff = pe.data();
            e.n_ex = nx.data(); e.n_ex_next = nn.data(); e.log_z_inc = lz.data();
            check(pf_estimate(b, &e), "estimate");
            for (uint32_t f = 0; f < cs.F; ++f) {
                const pf_master_t &r = traj[k * cs.F + f];
                bool ok = r.step == (uint64_t)(k + 1) && !memcmp(r.xhat, &xg[5 * f], 40) &&
                          !memcmp(&r.log_mass_glob, &lg[f], 8) && !memcmp(&r.pe_eff, &pe[f], 8) &&
                          !memcmp(&r.log_z_inc, &lz[f], 8) && r.n_ex == nx[f] && r.n_ex_next == nn[f];
                if (!ok) {
                    fprintf(stderr, "M=%u row %d filter %u differs\n", cs.M, k, f);
                    ++bad;
                }
            }
        }
        pf_destroy(a);
        pf_destroy(b);
        hipFree(traj);
        hipFree(d);
    }
    fprintf(stderr, bad ? "TRAJ MISMATCH\n" : "TRAJ EQUAL\n");
    return bad ? 2 : 0;
}

// One iteration of context c by k_step_flex with ppw PEs per workgroup of B
// threads, log-weights in LDS (ulds) or in u.
static int launch_flex(pf_ctx *c, const float *frame, float *u, uint32_t ppw, uint32_t B,
                       bool ulds) {
    const uint64_t k = c->step + 1;
    int rc = ensure_ring(c, k);
    if (rc != PF_OK) return rc;
    StepArgs a = make_args(c, k, frame);
    void *fn = pick_flex_kernel(c->half, c->cfg.lik_mode, ulds);
    double *lm = nullptr;
    void *args[] = {&a, &u, &ppw, &lm};
    const uint32_t grid = c->cfg.n_filters * ((c->cfg.n_pe + ppw - 1) / ppw);
    if (hipLaunchKernel(fn, dim3(grid), dim3(B), args,
                        flex_lds_bytes(ulds ? ppw * c->cfg.n_per_pe : 0, kSmallTile),
                        c->stream) != hipSuccess)
        return PF_EHIP;
    advance(c, k);
    return PF_OK;
}

template <class T>
static std::vector<T> dbg(pf_ctx *c, int which) {
    std::vector<T> v(pf_debug_size(c, which) / sizeof(T));
    check(pf_debug_get(c, which, v.data(), v.size() * sizeof(T)), "debug get");
    return v;
}

// Ancestors of one PE by systematic resampling, exact integer arithmetic:
// rank j goes to min { i : n C_i > j T + V }.
static std::vector<uint32_t> systematic(const uint32_t *q, uint32_t n, uint32_t V, uint64_t T) {
    std::vector<uint32_t> anc(n, 0);
    if (T == 0) return anc;
    uint64_t C = 0;
    uint32_t i = 0;
    for (uint32_t j = 0; j < n; ++j) {
        const uint64_t ptr = (uint64_t)j * T + V;
        while (i < n && (uint64_t)n * (C + q[i]) <= ptr) C += q[i++];
        anc[j] = i < n ? i : n - 1;
    }
    return anc;
}

// Iterations of context b (ppw = 0: through the library; else k_step_flex
// launched directly) against context a (through the library: k_step, or for
// PEs beyond the LDS stage the split kernels), both from the same state
// before every iteration: every traced value and the stored particles equal,
// the records within FP64 summation order.
static int compare_with_k_step(const Case &cs, uint32_t ppw_cfg, uint32_t block_cfg,
                               uint32_t ppw_direct, bool ulds, std::mt19937_64 &rng) {
    const int K = 5;
    Inputs in = make_inputs(cs, K, rng);
    float *d, *u;
    hipMalloc(&d, in.frames.size() * 4);
    memcpy(d, in.frames.data(), in.frames.size() * 4);
    pf_config cfg = make_cfg(cs);
    cfg.debug = PF_DEBUG_TRACE;
    pf_ctx *a, *b;
    check(pf_init(&cfg, in.truth.data(), &a), "init a");
    cfg.pes_per_wg = ppw_cfg;
    cfg.block_size = block_cfg;
    check(pf_init(&cfg, in.truth.data(), &b), "init b");
    hipMalloc(&u, b->N * 4);
    int diff = 0;
    double worst = 0;
    for (int k = 0; k < K; ++k) {
        check(launch_step(a, d + k * in.stride), "k_step");
        if (ppw_direct)
            check(launch_flex(b, d + k * in.stride, u, ppw_direct, 1024, ulds), "k_step_flex");
        else
            check(launch_step(b, d + k * in.stride), "k_step_flex via the library");
        hipDeviceSynchronize();
        const size_t N = a->N;
        diff += memcmp(a->prop[a->cur], b->prop[b->cur], 5 * N * 4) != 0;
        diff += memcmp(a->anc[a->cur], b->anc[b->cur], N * 2) != 0;
        const int exact[] = {PF_DBG_RING, PF_DBG_NEX, PF_DBG_SRC, PF_DBG_PROP, PF_DBG_ELL,
                             PF_DBG_Q, PF_DBG_ANCESTORS, PF_DBG_V, PF_DBG_LAMBDA};
        for (int w : exact) {
            std::vector<unsigned char> x = dbg<unsigned char>(a, w), y = dbg<unsigned char>(b, w);
            if (x != y) {
                fprintf(stderr, "np=%u step %d: debug buffer %d differs\n", cs.np, k, w);
                ++diff;
            }
        }
        for (uint64_t i = 0; i < a->FM; ++i) {
            const pf_pe_record &ra = a->rec[a->cur][i], &rb = b->rec[b->cur][i];
            diff += ra.lstar != rb.lstar || ra.total_q != rb.total_q;
            const double dl = fabs(ra.log_mass - rb.log_mass);
            worst = dl > worst ? dl : worst;
            diff += !(dl <= 1e-12 * (1 + fabs(ra.log_mass)));
            for (int c = 0; c < 5; ++c) {
                const double dx = fabs(ra.xhat[c] - rb.xhat[c]);
                worst = dx > worst ? dx : worst;
                diff += !(dx <= 1e-12 * (1 + fabs(ra.xhat[c])));
            }
        }
        if (a->mrec[0]) {   // the once-per-filter master records, within FP64 order
            for (uint32_t f = 0; f < cs.F; ++f) {
                const MasterRec &x = a->mrec[a->cur][f], &y = b->mrec[b->cur][f];
                diff += x.nex_next != y.nex_next ||
                        !(fabs(x.lglob - y.lglob) <= 1e-12 * (1 + fabs(x.lglob)));
            }
            memcpy(b->mrec[b->cur], a->mrec[a->cur], cs.F * sizeof(MasterRec));
        }
        // the next iteration starts from the same records
        memcpy(b->rec[b->cur], a->rec[a->cur], a->FM * sizeof(pf_pe_record));
    }
    fprintf(stderr, "F=%u M=%u np=%u lik=%u, %s ppw=%u block=%u: %s (largest record difference %.3g)\n",
            cs.F, cs.M, cs.np, cs.lik, ppw_direct ? (ulds ? "direct, u in LDS" : "direct, u in HBM")
                                                  : "library",
            ppw_direct ? ppw_direct : ppw_cfg, ppw_direct ? 1024 : b->block,
            diff ? "DIFFERENT" : "same", worst);
    pf_destroy(a);
    pf_destroy(b);
    hipFree(u);
    hipFree(d);
    return diff != 0;
}

static int stream_main() {
    int bad = 0;
    std::mt19937_64 rng(99);
    // (1) the streaming form (one PE per workgroup, log-weights in HBM) on
    // PEs k_step can run
    const Case same[] = {
        {1, 4, 256, 128, 128, 1, 0, 9, 0, 0, 0.1f, 5.f, 2.f, 1},
        {2, 3, 1000, 96, 80, 1, 0, 9, 0, 0, 0.1f, 5.f, 2.f, 2},
        {1, 3, 4096, 128, 128, 1, 2, 9, 0, 0, 0.1f, 10.f, 2.f, 3},
        {3, 2, 77, 128, 128, 0, 1, 9, 0, 0, 0.5f, 5.f, 1.f, 4},
        {1, 4, 3000, 64, 64, 1, 0, 5, 0, 0, 0.1f, 5.f, 2.f, 5},
        {1, 1, 2000, 64, 64, 1, 0, 9, 0, 0, 0.1f, 5.f, 2.f, 6},
    };
    for (const Case &cs : same) bad += compare_with_k_step(cs, 0, 0, 1, false, rng);
    // (2) several PEs per workgroup, through the library (pes_per_wg)
    struct Grouped { Case cs; uint32_t ppw, block; };
    const Grouped grouped[] = {
        {{1, 4, 256, 128, 128, 1, 0, 9, 0, 0, 0.1f, 5.f, 2.f, 21}, 2, 0},
        {{1, 4, 256, 128, 128, 1, 0, 9, 0, 0, 0.1f, 5.f, 2.f, 22}, 4, 512},
        {{3, 5, 77, 128, 128, 0, 1, 9, 0, 0, 0.5f, 5.f, 1.f, 23}, 3, 0},     // a partial last group
        {{2, 8, 300, 96, 80, 1, 0, 9, 0, 0, 0.1f, 5.f, 2.f, 24}, 8, 0},
        {{1, 6, 1000, 64, 48, 1, 2, 9, 0, 0, 0.1f, 10.f, 2.f, 25}, 4, 0},
        {{1, 3, 200, 64, 64, 1, 0, 7, 0, 0, 0.1f, 5.f, 2.f, 26}, 2, 0},
        {{1, 2100, 64, 96, 80, 1, 0, 9, 0, 0, 0.1f, 5.f, 2.f, 27}, 16, 0},  // master record
        {{2, 7, 130, 96, 80, 1, 0, 9, 0, 4, 0.1f, 5.f, 2.f, 28}, 5, 640},   // grouped ring
    };
    for (const Grouped &g : grouped) bad += compare_with_k_step(g.cs, g.ppw, g.block, 0, true, rng);
    // (3) contexts beyond the LDS stage: the library's split PEs (three
    // launches) against one streamed PE per workgroup, then through pf_step
    // against systematic resampling of the traced weights
    const Case big_cmp[] = {
        {1, 2, 5000, 128, 128, 1, 0, 9, 0, 0, 0.1f, 5.f, 2.f, 31},
        {2, 3, 8192, 96, 96, 0, 2, 9, 0, 0, 0.5f, 10.f, 2.f, 32},
        {1, 3, 4097, 64, 64, 1, 1, 9, 0, 0, 0.1f, 5.f, 1.f, 33},
        {1, 2, 20000, 128, 128, 1, 0, 9, 0, 0, 0.1f, 5.f, 2.f, 34},
    };
    for (const Case &cs : big_cmp) bad += compare_with_k_step(cs, 0, 0, 1, false, rng);
    const Case big[] = {
        {1, 2, 5000, 128, 128, 1, 0, 9, 0, 0, 0.1f, 5.f, 2.f, 11},
        {2, 3, 8192, 96, 96, 0, 2, 9, 1024, 0, 0.5f, 10.f, 2.f, 12},
        {1, 3, 4097, 64, 64, 1, 1, 9, 0, 0, 0.1f, 5.f, 1.f, 13},
        {1, 2, 65536, 128, 128, 1, 0, 9, 0, 0, 0.1f, 5.f, 2.f, 14},
    };
    for (const Case &cs : big) {
        const int K = 3;
        Inputs in = make_inputs(cs, K, rng);
        float *d;
        hipMalloc(&d, in.frames.size() * 4);
        memcpy(d, in.frames.data(), in.frames.size() * 4);
        pf_config cfg = make_cfg(cs);
        cfg.debug = PF_DEBUG_TRACE;
        pf_ctx *c;
        check(pf_init(&cfg, in.truth.data(), &c), "init big");
        int diff = 0;
        size_t distinct = 0;
        uint32_t nex = 0;
        for (int k = 0; k < K; ++k) {
            check(pf_step(c, d + k * in.stride), "step big");
            nex = dbg<uint32_t>(c, PF_DBG_NEX)[0];
            std::vector<uint32_t> q = dbg<uint32_t>(c, PF_DBG_Q), anc = dbg<uint32_t>(c, PF_DBG_ANCESTORS),
                                  v = dbg<uint32_t>(c, PF_DBG_V);
            std::vector<pf_pe_record> rec = dbg<pf_pe_record>(c, PF_DBG_PE_RECORDS);
            std::vector<uint16_t> a16(c->N);
            memcpy(a16.data(), c->anc[c->cur], c->N * 2);
            for (uint64_t pe = 0; pe < c->FM; ++pe) {
                const uint32_t *qp = q.data() + pe * cs.np;
                uint64_t T = 0;
                for (uint32_t i = 0; i < cs.np; ++i) T += qp[i];
                diff += T != rec[pe].total_q;
                const std::vector<uint32_t> want = systematic(qp, cs.np, v[pe], T);
                for (uint32_t j = 0; j < cs.np; ++j)
                    diff += want[j] != anc[pe * cs.np + j] || want[j] != a16[pe * cs.np + j];
                if (pe == 0) {
                    std::vector<uint32_t> w = want;
                    std::sort(w.begin(), w.end());
                    distinct = std::unique(w.begin(), w.end()) - w.begin();
                }
            }
        }
        fprintf(stderr, "np=%u M=%u lik=%u through pf_step: %s (last iteration: N_ex %u, "
                "%zu distinct ancestors in PE 0)\n", cs.np, cs.M, cs.lik,
                diff ? "WRONG ANCESTORS" : "ancestors exact", nex, distinct);
        bad += diff != 0;
        pf_destroy(c);
        hipFree(d);
    }
    fprintf(stderr, bad ? "STREAM MISMATCH\n" : "STREAM EQUAL\n");
    return bad ? 2 : 0;
}

// master_block, the in-kernel form of the master record, on the workgroup
// size of k_master.
__global__ void k_master_ref(const pf_pe_record *rec, MasterRec *out, uint32_t M, uint32_t np,
                             uint32_t mode, uint32_t fixed_nex, uint32_t cutoff_ppm) {
    __shared__ double red[kRedDoubles];
    master_block(rec + (size_t)blockIdx.x * M, M, np, mode, fixed_nex, cutoff_ppm, red,
                 out + blockIdx.x);
}

// k_master (every log-mass of a thread loaded before the reductions), from
// the records and from the compact log-masses (the latter also writing the
// master step's row), against master_block, bit for bit: random masses, PEs
// without mass, filters without mass, one PE holding it all; ragged M up to
// PF_MAX_PE.  The row against the master step in FP64 on the host.
static int master_main() {
    struct MC { uint32_t F, M, np, mode, kind; };
    const MC cases[] = {{1, 1, 64, 1, 0},     {2, 3, 100, 1, 1},    {1, 255, 4096, 1, 0},
                        {1, 256, 4096, 1, 1}, {3, 300, 77, 0, 0},   {1, 2100, 4, 1, 1},
                        {1, 8192, 128, 1, 0}, {2, 8192, 128, 1, 3}, {2, 600, 4100, 1, 2},
                        {1, 7999, 16, 1, 1}};
    std::mt19937_64 rng(5);
    std::normal_distribution<double> Nd(0, 3);
    std::uniform_int_distribution<int> coin(0, 3);
    int bad = 0;
    for (const MC &mc : cases) {
        const size_t n = (size_t)mc.F * mc.M;
        std::vector<pf_pe_record> rec(n);
        memset(rec.data(), 0, n * sizeof(pf_pe_record));
        for (size_t i = 0; i < n; ++i) {
            double L = Nd(rng);
            if (mc.kind == 1 && coin(rng) == 0) L = -INFINITY;   // PEs without mass
            if (mc.kind == 2) L = -INFINITY;                      // no mass at all
            if (mc.kind == 3) L = (i % mc.M == 17) ? 0.0 : -800.0;
            rec[i].log_mass = L;
            for (int c = 0; c < 5; ++c) rec[i].xhat[c] = 50.0 + 10.0 * Nd(rng);
        }
        pf_pe_record *d_rec;
        double *d_lm;
        MasterRec *d_a, *d_b, *d_c;
        pf_master_t *d_row;
        uint32_t *d_nex;
        hipMalloc(&d_row, mc.F * sizeof(pf_master_t));
        hipMalloc(&d_nex, mc.F * sizeof(uint32_t));
        for (uint32_t f = 0; f < mc.F; ++f) d_nex[f] = 7 + f;
        hipMalloc(&d_rec, n * sizeof(pf_pe_record));
        hipMalloc(&d_lm, n * sizeof(double));
        hipMalloc(&d_a, mc.F * sizeof(MasterRec));
        hipMalloc(&d_b, mc.F * sizeof(MasterRec));
        hipMalloc(&d_c, mc.F * sizeof(MasterRec));
        memcpy(d_rec, rec.data(), n * sizeof(pf_pe_record));
        for (size_t i = 0; i < n; ++i) d_lm[i] = rec[i].log_mass;
        memset(d_a, 0xAB, mc.F * sizeof(MasterRec));
        memset(d_b, 0xCD, mc.F * sizeof(MasterRec));
        memset(d_c, 0xEF, mc.F * sizeof(MasterRec));
        const uint32_t fixed_nex = mc.np / 10, cutoff = 990000;
        const double *no_lm = nullptr;
        // the library's choice of unrolling from the records, the widest one
        // from the compact log-masses
        check(launch_master(nullptr, mc.F, mc.M, mc.np, mc.mode, fixed_nex, cutoff, d_rec, no_lm,
                            d_a), "launch_master");
        hipLaunchKernelGGL(k_master<kMasterPerThread>, dim3(mc.F), dim3(kMasterThreads), 0,
                           nullptr, d_rec, (const double *)d_lm, d_c, d_row,
                           (const uint32_t *)d_nex, (uint64_t)42, mc.M, mc.np, mc.mode,
                           fixed_nex, cutoff);
        hipLaunchKernelGGL(k_master_ref, dim3(mc.F), dim3(kMasterThreads), 0, nullptr, d_rec, d_b,
                           mc.M, mc.np, mc.mode, fixed_nex, cutoff);
        hipDeviceSynchronize();
        bool eq = memcmp(d_a, d_b, mc.F * sizeof(MasterRec)) == 0 &&
                  memcmp(d_c, d_b, mc.F * sizeof(MasterRec)) == 0;
        for (uint32_t f = 0; f < mc.F; ++f) {   // the row, in FP64 on the host
            const pf_pe_record *R = rec.data() + (size_t)f * mc.M;
            double lmax = -INFINITY, W = 0, X[5] = {0, 0, 0, 0, 0};
            uint64_t S = 0, D = 0;
            for (uint32_t i = 0; i < mc.M; ++i) lmax = std::max(lmax, R[i].log_mass);
            for (uint32_t i = 0; lmax != -INFINITY && i < mc.M; ++i) {
                const double e = exp(R[i].log_mass - lmax);
                const uint64_t P = (uint64_t)floor(e * 1048576.0);
                W += e;
                S += P;
                D += P * P;
                for (int c = 0; e > 0.0 && c < 5; ++c) X[c] += e * R[i].xhat[c];
            }
            const pf_master_t &o = d_row[f];
            const double lg = lmax == -INFINITY ? -INFINITY : lmax + log(W);
            bool ok = o.step == 42 && o.n_ex == 7 + f && o.n_ex_next == d_b[f].nex_next &&
                      (o.log_mass_glob == d_b[f].lglob) &&
                      (lmax == -INFINITY ? o.log_mass_glob == -INFINITY
                                         : fabs(o.log_mass_glob - lg) <= 1e-12 * (1 + fabs(lg))) &&
                      o.pe_eff == (D ? (double)S * (double)S / (double)D : 0.0);
            for (int c = 0; lmax != -INFINITY && c < 5; ++c)
                ok = ok && fabs(o.xhat[c] - X[c] / W) <= 1e-12 * (1 + fabs(X[c] / W));
            if (!ok)
                fprintf(stderr, "  row of filter %u: log W %.17g / %.17g, PE_eff %.17g, x %.17g / %.17g\n",
                        f, o.log_mass_glob, lg, o.pe_eff, o.xhat[0], X[0] / W);
            eq = eq && ok;
        }
        fprintf(stderr, "master F=%u M=%u np=%u mode=%u kind=%u: %s (log W %.17g, N_ex %u)\n",
                mc.F, mc.M, mc.np, mc.mode, mc.kind, eq ? "equal" : "DIFFERENT", d_a[0].lglob,
                d_a[0].nex_next);
        bad += !eq;
        hipFree(d_rec);
        hipFree(d_lm);
        hipFree(d_a);
        hipFree(d_b);
        hipFree(d_c);
        hipFree(d_row);
        hipFree(d_nex);
    }
    fprintf(stderr, bad ? "MASTER MISMATCH\n" : "MASTER EQUAL\n");
    return bad ? 2 : 0;
}

int main(int argc, char **argv) {
    if (argc > 1 && !strcmp(argv[1], "batch")) {
        if (argc > 4) emu_set_fill(atoi(argv[4]));
        return batch_main(argc > 2 ? atoi(argv[2]) : 70, argc > 3 ? atoi(argv[3]) : 0);
    }
    if (argc > 1 && !strcmp(argv[1], "traj")) return traj_main();
    if (argc > 1 && !strcmp(argv[1], "stream")) return stream_main();
    if (argc > 1 && !strcmp(argv[1], "master")) return master_main();
    fprintf(stderr, "usage: %s batch K MODE [FILL] | traj | stream | master\n", argv[0]);
    return 1;
}
