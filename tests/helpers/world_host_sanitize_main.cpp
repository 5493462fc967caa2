// Drives the host-side code of libworld that touches no device (configuration
// checks, arena layout and sizes, regrowth thresholds, image validation,
// argument checks of world_create) under AddressSanitizer and
// UndefinedBehaviorSanitizer.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "world.h"

#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            std::exit(1);                                                 \
        }                                                                 \
    } while (0)

static world_config base(int H, int W, int cap, int n0, int rho, int hd) {
    world_config c;
    std::memset(&c, 0, sizeof(c));
    c.struct_size = sizeof(c);
    c.H = H; c.W = W; c.cap = cap; c.n_init = n0; c.obs_radius = rho; c.hidden = hd;
    c.res_init_p = 0.3; c.rate_bottom = 0.02; c.rate_top = 0.002; c.rate_scale = 5.0; c.spont = 1e-5;
    c.E0 = 50; c.decay = 1; c.gain = 10; c.E_repr = 40; c.T_repr = 20; c.L_max = 2000;
    c.sigma_mut = 0.02; c.w_init_gain = 0.5; c.regrow_alpha = 1.0;
    return c;
}

struct Img {
    std::vector<uint8_t> R, la, ate;
    std::vector<uint32_t> uid;
    std::vector<int32_t> row, col, e, age, st;
    std::vector<float> h, theta;
    world_image im;
    Img(const world_config& c, int n, int P, int ss) {
        R.assign(size_t(c.H) * c.W, 0);
        la.assign(n + 1, 5); ate.assign(n + 1, 0); uid.resize(n + 1); row.resize(n + 1); col.resize(n + 1);
        e.assign(n + 1, 50); age.assign(n + 1, 0); st.assign(n + 1, 0);
        h.assign(size_t(n + 1) * ss, 0.f); theta.assign(size_t(n + 1) * P, 0.f);
        for (int i = 0; i < n; ++i) {
            uid[i] = 3 * i;
            row[i] = i / c.W;
            col[i] = i % c.W;
        }
        std::memset(&im, 0, sizeof(im));
        im.struct_size = sizeof(im);
        im.flags = WORLD_SNAP_HIDDEN | WORLD_SNAP_THETA;
        im.n_live = n;
        im.next_uid = 3 * n;
        im.agent_capacity = n;
        im.R = R.data(); im.uid = uid.data(); im.row = row.data(); im.col = col.data(); im.energy = e.data();
        im.age = age.data(); im.streak = st.data(); im.h = h.data(); im.theta = theta.data();
        im.last_action = la.data(); im.ate = ate.data();
    }
};

int main() {
    std::vector<world_config> good = {base(32, 64, 256, 32, 2, 16), base(200, 400, 4608, 4096, 3, 32),
                                      base(200, 400, 16384, 12000, 3, 32), base(2, 1, 1, 1, 1, 16)};
    world_config net = base(200, 400, 1000, 330, 7, 4);
    net.controller = WORLD_CTRL_CNN_LSTM;
    net.dynamics = WORLD_DYN_PAPER; net.E0 = 120; net.E_max = 120; net.T_death = 200; net.regrow_pI = 0.002;
    net.regrow_alpha = 200.0;
    good.push_back(net);
    for (const world_config& c : good) {
        size_t dev = 0, snap = 0;
        CHECK(world_required_bytes(&c, &dev, &snap) == WORLD_OK && dev > 0 && snap > 0);
        int32_t n_in = 0, P = 0;
        CHECK(world_dims(&c, &n_in, &P) == WORLD_OK && n_in > 0 && P > 0);
        std::vector<uint64_t> thr(size_t(c.H) * 25);
        CHECK(world_threshold_table(&c, thr.data()) == WORLD_OK);
        const int ss = c.controller == WORLD_CTRL_CNN_LSTM ? 8 : c.hidden;
        const int n = c.n_init < c.H * c.W ? c.n_init : c.H * c.W;
        Img ok(c, n, P, ss);
        CHECK(world_validate_image(&c, &ok.im) == WORLD_OK);
        if (n >= 2) {
            Img bad(c, n, P, ss);
            bad.uid[1] = bad.uid[0];
            CHECK(world_validate_image(&c, &bad.im) == WORLD_E_INVALID_ARG);
            Img out(c, n, P, ss);
            out.row[n - 1] = c.H;
            CHECK(world_validate_image(&c, &out.im) == WORLD_E_INVALID_ARG);
            Img two(c, n, P, ss);
            two.row[1] = two.row[0];
            two.col[1] = two.col[0];
            CHECK(world_validate_image(&c, &two.im) ==
                  (c.dynamics == WORLD_DYN_PAPER ? WORLD_OK : WORLD_E_INVALID_ARG));
        }
        Img res(c, n, P, ss);
        res.R[0] = 2;
        CHECK(world_validate_image(&c, &res.im) == WORLD_E_INVALID_ARG);
        Img big(c, 0, P, ss);
        big.im.n_live = c.cap + 1;
        CHECK(world_validate_image(&c, &big.im) == WORLD_E_INVALID_ARG);
        Img part(c, n, P, ss);
        part.im.flags = WORLD_SNAP_HIDDEN;
        CHECK(world_validate_image(&c, &part.im) == WORLD_E_INVALID_ARG);
        // creation rejects a misaligned or short arena before any device call
        std::vector<uint8_t> fake(256 + 64);
        world_t* w = nullptr;
        uint8_t* mis = fake.data() + ((reinterpret_cast<uintptr_t>(fake.data()) % 256) == 1 ? 2 : 1);
        CHECK(world_create(&c, 7, mis, dev, nullptr, &w) == WORLD_E_INVALID_ARG && w == nullptr);
    }
    world_config bad = base(1, 10, 16, 4, 2, 16);
    size_t dev = 0;
    CHECK(world_required_bytes(&bad, &dev, nullptr) == WORLD_E_INVALID_CONFIG);
    bad = base(10, 10, 16, 40, 2, 16);
    CHECK(world_required_bytes(&bad, &dev, nullptr) == WORLD_E_INVALID_CONFIG);
    bad = base(10, 10, 16, 4, 2, 24);
    CHECK(world_dims(&bad, nullptr, nullptr) == WORLD_E_INVALID_CONFIG);
    CHECK(world_validate_image(&good[0], nullptr) == WORLD_E_INVALID_ARG);
    CHECK(world_last_error(nullptr)[0] != 0);
    std::puts("ok");
    return 0;
}
