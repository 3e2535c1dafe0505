// Exercises the host side of libstencil (plan creation and validation,
// option checks, dispatch-map and tuning-cache parsing, workspace sizes,
// coefficient reports, batched plans, and every argument check that
// returns before device work) in a build with AddressSanitizer and
// UndefinedBehaviorSanitizer; made and run by tests/test_sanitizers.py
// without a GPU.  Prints "ok" on success.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "stencil.h"

#define EXPECT(cond)                                                         \
    do {                                                                     \
        if (!(cond)) {                                                       \
            fprintf(stderr, "failed: %s (line %d): %s\n", #cond, __LINE__,   \
                    stencil_last_error());                                   \
            return 1;                                                        \
        }                                                                    \
    } while (0)

static st_problem prob(int ndim, long nx, long ny, long nz, int shape, int r, const float* c, int dtype,
                       int bc, int update) {
    st_problem p;
    memset(&p, 0, sizeof p);
    p.ndim = ndim;
    p.n[0] = nx;
    p.n[1] = ny;
    p.n[2] = nz;
    p.shape = shape;
    p.radius = r;
    p.coeffs = c;
    p.dtype = dtype;
    p.boundary = bc;
    p.update = update;
    return p;
}

int main(int argc, char** argv) {
    std::vector<float> c(729, 0.f);
    for (int i = 0; i < 729; ++i) c[i] = 0.001f * (float)(i % 7);
    std::vector<float> star(729, 0.f);
    // 2D and 3D linear plans over shapes, radii, dtypes and boundaries
    for (int ndim = 2; ndim <= 3; ++ndim)
        for (int shape = 0; shape < 2; ++shape)
            for (int r = 1; r <= 4; ++r)
                for (int dtype = 0; dtype < 3; ++dtype)
                    for (int bc = 0; bc < 2; ++bc) {
                        const int w = 2 * r + 1, cnt = ndim == 3 ? w * w * w : w * w;
                        std::vector<float> cc(cnt, 0.f);
                        for (int i = 0; i < cnt; ++i) {
                            const int dx = i % w - r, dy = (i / w) % w - r, dz = ndim == 3 ? i / (w * w) - r : 0;
                            if (shape == 1 || (dz != 0) + (dy != 0) + (dx != 0) <= 1) cc[i] = 0.01f;
                        }
                        st_problem p = prob(ndim, 300, 200, ndim == 3 ? 40 : 1, shape, r, cc.data(), dtype, bc, 0);
                        st_plan* h = nullptr;
                        const st_status s = stencil_plan(&p, nullptr, &h);
                        if (shape == 1 && r > 2) {
                            EXPECT(s == ST_EUNSUPPORTED && h == nullptr);
                            continue;
                        }
                        EXPECT(s == ST_OK);
                        int32_t v, tx, ty, k, zc;
                        EXPECT(stencil_plan_describe(h, &v, &tx, &ty, &k, &zc) == ST_OK);
                        EXPECT(stencil_workspace_bytes(h, 5, 0) > 0);
                        (void)stencil_workspace_bytes(h, 0, 2);
                        std::vector<float> back(cnt + 3, -1.f);
                        double sum = 0;
                        EXPECT(stencil_plan_coefficients(h, back.data(), cnt + 3, &sum) == ST_OK);
                        EXPECT(back[cnt] == -1.f);   // wrote no more than the plan holds
                        int fake = 0;
                        EXPECT(stencil_apply(h, &fake, &fake, -1, nullptr, nullptr, 0, nullptr) == ST_EINVAL);
                        EXPECT(stencil_apply(h, &fake, &fake + 1, 3, nullptr, nullptr, 0, nullptr) == ST_EWORKSPACE);
                        EXPECT(stencil_apply_noalloc(h, &fake, &fake, -2, nullptr, nullptr) == ST_EINVAL);
                        stencil_plan_destroy(h);
                    }
    // options
    {
        st_problem p = prob(2, 256, 256, 1, 0, 1, c.data(), 0, 0, 0);
        std::vector<float> cc(9, 0.f);
        cc[1] = cc[3] = cc[4] = cc[5] = cc[7] = 0.2f;
        p.coeffs = cc.data();
        st_plan_opts o{1, 4, 16, 1, 0, 0};
        st_plan* h = nullptr;
        EXPECT(stencil_plan(&p, &o, &h) == ST_EINVAL);
        o = st_plan_opts{5, 256, 0, 2, 0, 0};
        EXPECT(stencil_plan(&p, &o, &h) == ST_OK);
        stencil_plan_destroy(h);
        o = st_plan_opts{0, 0, 0, 0, 0, -3};
        EXPECT(stencil_plan(&p, &o, &h) == ST_EINVAL);
        cc[0] = 1.f;   // off the star
        EXPECT(stencil_plan(&p, nullptr, &h) == ST_EINVAL);
    }
    // wave plans: workspaces, gradient layout, coefficients, argument and layer checks
    {
        st_problem p = prob(3, 48, 40, 36, 0, 4, nullptr, 0, 1, 1);
        st_plan_opts o{0, 0, 0, 0, 0, 7};
        st_plan* h = nullptr;
        EXPECT(stencil_plan(&p, &o, &h) == ST_OK);
        EXPECT(stencil_workspace_bytes(h, 30, 1) > stencil_workspace_bytes(h, 30, 0));
        double sum = 1.0;
        EXPECT(stencil_plan_coefficients(h, nullptr, 0, &sum) == ST_OK && sum == 0.0);
        int fake = 0;
        st_wave_args wa;
        memset(&wa, 0, sizeof wa);
        wa.u_prev = (void*)0x3000;
        wa.kappa = (const float*)0x4000;
        wa.src[0] = -1;
        wa.rec_z = -1;
        wa.sponge_width = 30;   // wider than half the grid
        wa.sponge_strength = 0.5f;
        EXPECT(stencil_apply(h, &fake, &fake + 1, 2, &wa, nullptr, 0, nullptr) == ST_EINVAL);
        wa.sponge_width = 4;
        wa.sponge_strength = -1.f;
        EXPECT(stencil_apply_adjoint(h, &fake, &fake + 1, 2, &wa, nullptr, 0, nullptr) == ST_EINVAL);
        wa.sponge_strength = 0.5f;
        wa.src[0] = 100;
        EXPECT(stencil_apply(h, &fake, &fake + 1, 2, &wa, nullptr, 0, nullptr) == ST_EINVAL);
        wa.src[0] = -1;
        wa.rec_z = 2;
        EXPECT(stencil_wave_gradient(h, &fake, &wa, 5, (float*)0x5000, (double*)0x6000, nullptr, 0, nullptr) ==
               ST_EINVAL);   // no target
        stencil_plan_destroy(h);
        p.boundary = 0;
        EXPECT(stencil_plan(&p, nullptr, &h) == ST_OK);
        wa.rec_z = -1;
        EXPECT(stencil_apply(h, &fake, &fake + 1, 2, &wa, nullptr, 0, nullptr) == ST_EUNSUPPORTED);
        stencil_plan_destroy(h);
        p.dtype = 1;
        EXPECT(stencil_plan(&p, nullptr, &h) == ST_EUNSUPPORTED);
    }
    // variable coefficients
    {
        st_problem p = prob(3, 40, 30, 20, 1, 1, nullptr, 0, 0, 2);
        st_plan* h = nullptr;
        EXPECT(stencil_plan(&p, nullptr, &h) == ST_OK);
        int fake = 0;
        EXPECT(stencil_apply_varcoef(h, &fake, &fake, nullptr, 1, nullptr, 0, nullptr) == ST_EINVAL);
        EXPECT(stencil_apply(h, &fake, &fake, 1, nullptr, nullptr, 0, nullptr) == ST_EINVAL);
        stencil_plan_destroy(h);
    }
    // batched plans
    {
        std::vector<float> cc(25, 0.04f);
        std::vector<st_problem> ps;
        for (int i = 0; i < 9; ++i) ps.push_back(prob(2, 64 + 37 * i, 50 + 11 * i, 1, 1, 2, cc.data(), 0, i % 2 ? 0 : 0, 0));
        st_plan* h = nullptr;
        EXPECT(stencil_plan_batched(ps.data(), (int)ps.size(), nullptr, &h) == ST_OK);
        EXPECT(stencil_workspace_bytes(h, 8, 0) > 0);
        (void)stencil_workspace_bytes(h, 0, 2);
        int32_t tried, rejected;
        EXPECT(stencil_autotune_stats(h, &tried, &rejected) == ST_OK);
        std::vector<void*> ptrs(9, (void*)0x1000);
        EXPECT(stencil_apply_batched(h, ptrs.data(), ptrs.data(), 8, nullptr, 0, nullptr) == ST_EWORKSPACE);
        EXPECT(stencil_apply_batched(h, ptrs.data(), ptrs.data(), -1, nullptr, 0, nullptr) == ST_EINVAL);
        EXPECT(stencil_plan_coefficients(h, nullptr, 0, nullptr) == ST_EINVAL);
        // The launch schedule (member tables built and checked on the host)
        // at a batch depth and at each member's own depth.
        for (int steps : {1, 7, 32}) {
            int32_t launches = 0, tables = 0;
            int64_t wg = 0;
            EXPECT(stencil_plan_describe_batched(h, steps, 256, &launches, &tables, &wg) == ST_OK);
            EXPECT(launches >= 1 && tables >= 1 && wg >= launches);
        }
        EXPECT(stencil_plan_describe_batched(h, 0, 256, nullptr, nullptr, nullptr) == ST_EINVAL);
        stencil_plan_destroy(h);
        st_plan_opts own;
        memset(&own, 0, sizeof own);
        own.tsteps = -1;
        EXPECT(stencil_plan_batched(ps.data(), (int)ps.size(), &own, &h) == ST_OK);
        for (int steps : {1, 5, 33}) EXPECT(stencil_plan_describe_batched(h, steps, 7, nullptr, nullptr, nullptr) == ST_OK);
        stencil_plan_destroy(h);
        own.tsteps = -2;
        EXPECT(stencil_plan_batched(ps.data(), (int)ps.size(), &own, &h) == ST_EINVAL);
        ps[3].dtype = 1;
        EXPECT(stencil_plan_batched(ps.data(), (int)ps.size(), nullptr, &h) == ST_EINVAL);
        EXPECT(stencil_plan_batched(ps.data(), 0, nullptr, &h) == ST_EINVAL);
    }
    EXPECT(stencil_plan(nullptr, nullptr, nullptr) == ST_EINVAL);
    stencil_plan_destroy(nullptr);
    EXPECT(strstr(stencil_version(), "gfx950") != nullptr);
    printf("ok\n");
    (void)argc;
    (void)argv;
    return 0;
}
