// C ABI of libqnep (declared in include/qnep.h): validation, workspace layout and
// the launch sequence of one qNEP evaluation on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>

#include "plan.h"

namespace qnep {
bool nep_supported(int T, int NR, int NA, int NBR, int NBA, int LMAX);
hipError_t launch_phi_mean(const Plan &p);
bool mlp_bf16_supported(int ndes, int H);
int radial_table_row(int NB);
}  // namespace qnep

using namespace qnep;

namespace {

thread_local std::string g_last_error;

qnep_status fail(qnep_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

const char *const kStageNames[QNEP_N_STAGES] = {
    "sort", "lists", "lists_coulomb", "descriptors", "mlp", "real_space", "ewald_structure_factor",
    "ewald_atoms", "pppm_spread", "fft_forward", "pppm_influence", "fft_inverse", "pppm_gather", "phi_mean",
    "radial_forces", "angular_forces_energy", "angular_forces_charge", "assemble", "finalize", "other"};

}  // namespace

namespace qnep {
// Ring of per-call HIP event sets; a full ring drains its oldest call.
struct Timer {
    static constexpr int SLOTS = 64, MARKS = 40;
    bool on = false;
    hipEvent_t ev[SLOTS][MARKS];
    int ids[SLOTS][MARKS];
    int nl[SLOTS][MARKS];
    int nm[SLOTS];
    int head = 0, count = 0, cur = -1;
    double total[QNEP_N_STAGES] = {0};
    int64_t launches[QNEP_N_STAGES] = {0};
    int calls = 0;
    bool created = false;

    hipError_t create() {
        if (created) return hipSuccess;
        for (int s = 0; s < SLOTS; ++s)
            for (int m = 0; m < MARKS; ++m) {
                hipError_t e = hipEventCreate(&ev[s][m]);
                if (e != hipSuccess) return e;
            }
        created = true;
        return hipSuccess;
    }
    void destroy() {
        if (!created) return;
        for (int s = 0; s < SLOTS; ++s)
            for (int m = 0; m < MARKS; ++m) (void)hipEventDestroy(ev[s][m]);
        created = false;
    }
    hipError_t drain_one() {
        const int s = head;
        if (nm[s] > 1) {
            hipError_t e = hipEventSynchronize(ev[s][nm[s] - 1]);
            if (e != hipSuccess) return e;
            for (int m = 1; m < nm[s]; ++m) {
                float ms = 0.f;
                e = hipEventElapsedTime(&ms, ev[s][m - 1], ev[s][m]);
                if (e != hipSuccess) return e;
                total[ids[s][m]] += ms;
                launches[ids[s][m]] += nl[s][m];
            }
        }
        ++calls;
        head = (head + 1) % SLOTS;
        --count;
        return hipSuccess;
    }
    hipError_t begin(hipStream_t st) {
        if (count == SLOTS) {
            hipError_t e = drain_one();
            if (e != hipSuccess) return e;
        }
        cur = (head + count) % SLOTS;
        ++count;
        nm[cur] = 0;
        return mark(st, ST_OTHER, 0);
    }
    hipError_t mark(hipStream_t st, int id, int n) {
        if (cur < 0 || nm[cur] >= MARKS) return hipSuccess;
        ids[cur][nm[cur]] = id;
        nl[cur][nm[cur]] = n;
        return hipEventRecord(ev[cur][nm[cur]++], st);
    }
};

void stage_mark(const Plan &p, int stage, int launches) {
    if (p.timer && p.timer->on) (void)p.timer->mark(p.stream, stage, launches);
}
}  // namespace qnep

namespace {

struct Model {
    qnep_hparams hp;
    int prec;
    double cap_factor;
    Timer timer;
};

constexpr size_t ALIGN = 256;

struct Carver {
    char *base;
    size_t off = 0;
    bool dry;
    template <class T>
    T *take(size_t count) {
        off = (off + ALIGN - 1) / ALIGN * ALIGN;
        T *p = dry ? nullptr : reinterpret_cast<T *>(base + off);
        off += sizeof(T) * (count > 0 ? count : 1);
        return p;
    }
};

bool invert_cell(const double *h, double *hi, double *vol) {
    double d = h[0] * (h[4] * h[8] - h[5] * h[7]) - h[1] * (h[3] * h[8] - h[5] * h[6]) +
               h[2] * (h[3] * h[7] - h[4] * h[6]);
    if (!(d > 1e-9)) return false;  // singular or left-handed
    hi[0] = (h[4] * h[8] - h[5] * h[7]) / d;
    hi[1] = (h[2] * h[7] - h[1] * h[8]) / d;
    hi[2] = (h[1] * h[5] - h[2] * h[4]) / d;
    hi[3] = (h[5] * h[6] - h[3] * h[8]) / d;
    hi[4] = (h[0] * h[8] - h[2] * h[6]) / d;
    hi[5] = (h[2] * h[3] - h[0] * h[5]) / d;
    hi[6] = (h[3] * h[7] - h[4] * h[6]) / d;
    hi[7] = (h[1] * h[6] - h[0] * h[7]) / d;
    hi[8] = (h[0] * h[4] - h[1] * h[3]) / d;
    *vol = d;
    return true;
}

void cell_widths(const double *h, double vol, double *w) {
    for (int a = 0; a < 3; ++a) {
        const double *u = h + 3 * ((a + 1) % 3), *v = h + 3 * ((a + 2) % 3);
        double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2], cz = u[0] * v[1] - u[1] * v[0];
        w[a] = vol / std::sqrt(cx * cx + cy * cy + cz * cz);
    }
}

int64_t param_count(const qnep_hparams &hp) {
    int64_t T = hp.n_types;
    int64_t ndes = (hp.n_max_R + 1) + (int64_t)(hp.n_max_A + 1) * hp.l_max;
    return T * T * (hp.n_max_R + 1) * (hp.basis_R + 1) + T * T * (hp.n_max_A + 1) * (hp.basis_A + 1) +
           T * (hp.n_neu * ndes + 3 * hp.n_neu + 1) + 2;
}

int capacity(double density, double rc, double factor) {
    double mean = density * 4.0 / 3.0 * M_PI * rc * rc * rc;
    int cap = (int)std::ceil(factor * mean + 32.0);
    return (cap + 7) / 8 * 8;
}

// Host-side exact count of the half set of wave vectors (same rule as the device).
int64_t count_half_k(const double *hi, int M0, int M1, int M2, double kmax, int inclusive) {
    int64_t n = 0;
    double km2 = kmax * kmax;
    for (int a2 = 0; a2 <= M2; ++a2)
        for (int a1 = -M1; a1 <= M1; ++a1)
            for (int a0 = -M0; a0 <= M0; ++a0) {
                bool half = a2 > 0 || (a2 == 0 && (a1 > 0 || (a1 == 0 && a0 > 0)));
                if (!half) continue;
                double kx = 2.0 * M_PI * (hi[0] * a0 + hi[1] * a1 + hi[2] * a2);
                double ky = 2.0 * M_PI * (hi[3] * a0 + hi[4] * a1 + hi[5] * a2);
                double kz = 2.0 * M_PI * (hi[6] * a0 + hi[7] * a1 + hi[8] * a2);
                double k2 = kx * kx + ky * ky + kz * kz;
                bool keep = inclusive ? (k2 <= km2 * (1.0 + 1e-9)) : (k2 < km2 * (1.0 - 1e-9));
                n += keep ? 1 : 0;
            }
    return n;
}

// Fills every size field of the plan and carves the workspace (dry run when base is null).
qnep_status make_plan(const Model &m, const qnep_es_params *es, const qnep_system *sys, char *base, Plan &p,
                      size_t *bytes, bool backward = false) {
    const qnep_hparams &hp = m.hp;
    if (!es || !sys) return fail(QNEP_E_INVALID_ARG, "null es or system");
    if (sys->n_atoms < 0 || sys->n_atoms >= (int64_t)(1u << IDX_BITS))
        return fail(QNEP_E_INVALID_ARG, "n_atoms must be in [0, 2^23)");
    p.N = (int)sys->n_atoms;
    p.T = hp.n_types;
    p.NR = hp.n_max_R + 1;
    p.NA = hp.n_max_A + 1;
    p.NBR = hp.basis_R + 1;
    p.NBA = hp.basis_A + 1;
    p.LMAX = hp.l_max;
    p.H = hp.n_neu;
    p.ndes = p.NR + p.NA * p.LMAX;
    p.rcR = hp.rc_R;
    p.rcA = hp.rc_A;
    p.mlp_prec = m.prec;
    p.off_cR = 0;
    p.off_cA = (int64_t)p.T * p.T * p.NR * p.NBR;
    p.off_nn = p.off_cA + (int64_t)p.T * p.T * p.NA * p.NBA;
    p.per_species = (int64_t)p.H * p.ndes + 3 * p.H + 1;
    p.off_b1E = p.off_nn + p.T * p.per_species;
    p.off_s = p.off_b1E + 1;
    p.n_theta = p.off_s + 1;
    if (es->mode != 1 && es->mode != 2) return fail(QNEP_E_INVALID_ARG, "mode must be 1 or 2");
    if (es->method != 0 && es->method != 1) return fail(QNEP_E_INVALID_ARG, "method must be 0 (Ewald) or 1 (PPPM)");
    if (!(es->alpha > 0)) return fail(QNEP_E_INVALID_ARG, "alpha must be positive");
    if (es->mode == 1 && !(es->rc_coul > 0)) return fail(QNEP_E_INVALID_ARG, "rc_coul must be positive");
    p.mode = es->mode;
    p.method = es->method;
    p.alpha = es->alpha;
    p.rc_coul = es->rc_coul;
    p.kmax = es->kmax;
    p.kinc = es->kmax_inclusive ? 1 : 0;
    p.order = es->order;
    p.qtot = es->q_total;
    for (int a = 0; a < 3; ++a) p.mesh[a] = es->mesh[a];
    std::memcpy(p.cell.h, sys->cell, sizeof(double) * 9);
    if (!invert_cell(p.cell.h, p.cell.hinv, &p.vol))
        return fail(QNEP_E_INVALID_ARG, "cell must be non-singular and right-handed");
    double w[3];
    cell_widths(p.cell.h, p.vol, w);
    const double rbin = 0.5 * std::max(p.rcR, p.rcA);
    for (int a = 0; a < 3; ++a) {
        p.nc[a] = std::max(1, (int)std::floor(w[a] / rbin));
        p.mR[a] = (int)std::ceil(std::max(p.rcR, p.rcA) * p.nc[a] / w[a] - 1e-12);
        p.mC[a] = (int)std::ceil(p.rc_coul * p.nc[a] / w[a] - 1e-12);
        if (p.mR[a] < 1) p.mR[a] = 1;
        if (p.mC[a] < 1) p.mC[a] = 1;
        if (p.mR[a] > 3 * p.nc[a] || (p.mode == 1 && p.mC[a] > 3 * p.nc[a]))
            return fail(QNEP_E_UNSUPPORTED, "cell thinner than a third of a cutoff along an axis");
    }
    p.ncell = p.nc[0] * p.nc[1] * p.nc[2];
    const double density = p.N / p.vol;
    p.capR = capacity(density, p.rcR, m.cap_factor);
    p.capA = capacity(density, p.rcA, m.cap_factor);
    p.nblk = (p.N + RED_THREADS - 1) / RED_THREADS;
    int64_t red_blocks = std::max(p.nblk, 1);
    if (p.method == 0) {
        if (!(p.kmax > 0)) return fail(QNEP_E_INVALID_ARG, "kmax must be positive for Ewald");
        for (int a = 0; a < 3; ++a) {
            const double *v = p.cell.h + 3 * a;
            double len = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            p.nk_box[a] = (int)std::floor(p.kmax * len / (2.0 * M_PI)) + 1;
        }
        int64_t nh = count_half_k(p.cell.hinv, p.nk_box[0], p.nk_box[1], p.nk_box[2], p.kmax, p.kinc);
        p.nk_cap = nh + 16;
        p.s_chunks = std::max(1, (p.N + 511) / 512);
        red_blocks = std::max<int64_t>(red_blocks, (p.nk_cap + 255) / 256);
    } else {
        if (p.order != 5) return fail(QNEP_E_UNSUPPORTED, "PPPM assignment order must be 5");
        for (int a = 0; a < 3; ++a)
            if (!fft_length_supported(p.mesh[a]))
                return fail(QNEP_E_UNSUPPORTED, "mesh sizes must be products of 2, 3, 5 up to 1024");
        p.mesh_pts = (int64_t)p.mesh[0] * p.mesh[1] * p.mesh[2];
        red_blocks = std::max<int64_t>(red_blocks, (p.mesh_pts + 255) / 256);
        // bricks of bins for the atomic-free spread: the first shape whose LDS tile
        // (B N / nc + 8 points per axis) fits 12288 floats
        static const int shapes[][3] = {{4, 4, 8}, {4, 4, 6}, {4, 4, 4}, {3, 3, 4}, {2, 2, 4}, {2, 2, 2}, {1, 1, 2},
                                        {1, 1, 1}};
        for (const auto &sh : shapes) {
            int T[3], B[3];
            int64_t vol = 1;
            for (int a = 0; a < 3; ++a) {
                B[a] = std::min(sh[a], p.nc[a]);
                T[a] = (int)(((int64_t)B[a] * p.mesh[a] + p.nc[a] - 1) / p.nc[a]) + 8;
                vol *= T[a];
            }
            if (vol <= 12288) {
                for (int a = 0; a < 3; ++a) {
                    p.tileB[a] = B[a];
                    p.tileT[a] = T[a];
                    p.tileNb[a] = (p.nc[a] + B[a] - 1) / B[a];
                }
                break;
            }
        }
    }
    p.partials_cap = red_blocks * 11;
    const int64_t N = std::max(p.N, 1);
    Carver c{base, 0, base == nullptr};
    p.flags = c.take<int32_t>(16);
    p.scalars = c.take<double>(64);
    p.partials = c.take<double>(p.partials_cap);
    p.cid = c.take<int>(N);
    p.cell_count = c.take<int>(p.ncell);
    p.cell_start = c.take<int>(p.ncell + 1);
    p.cell_cursor = c.take<int>(p.ncell);
    p.scan_tmp = c.take<int>((p.ncell + 1023) / 1024 + 1);
    p.perm = c.take<int>(N);
    p.xyzt = c.take<float4>(N);
    p.ts = c.take<int>(N);
    p.listR = c.take<uint32_t>((size_t)p.capR * N);
    p.cntR = c.take<int>(N);
    p.listA = c.take<uint32_t>((size_t)p.capA * N);
    p.cntA = c.take<int>(N);
    p.D = c.take<float>((size_t)p.ndes * N);
    p.Amom = c.take<float>((size_t)p.NA * LM * N);
    p.U = c.take<float>(N);
    p.qraw = c.take<float>(N);
    p.gU = c.take<float>((size_t)p.ndes * N);
    p.gq = c.take<float>((size_t)p.ndes * N);
    p.phi = c.take<float>(N);
    p.Fst = c.take<float>(3 * (size_t)N);
    p.hT = c.take<float>((size_t)2 * p.T * radial_table_row(p.NBR) * N);
    p.pairF = c.take<float>((size_t)4 * p.capA * N);
    p.pairA = c.take<float>((size_t)4 * p.capA * N);
    p.Fnep = c.take<float>(3 * (size_t)N);
    p.Znep = c.take<float>(9 * (size_t)N);
    if (p.method == 0) {
        p.kvec = c.take<float4>(2 * (size_t)p.nk_cap);  // kv then kn (int4)
        p.kcount = c.take<int>(1);
        p.Spart = c.take<float2>((size_t)p.s_chunks * p.nk_cap);
        p.Sk = c.take<float2>(p.nk_cap);
    } else {
        if (p.tileB[0] > 0) {
            const size_t nbricks = (size_t)p.tileNb[0] * p.tileNb[1] * p.tileNb[2];
            p.tiles = c.take<float>(nbricks * p.tileT[0] * p.tileT[1] * p.tileT[2]);
        } else {
            p.rho = c.take<float>(p.mesh_pts);
        }
        p.meshA = c.take<float2>(p.mesh_pts);
        p.meshB = c.take<float2>(p.mesh_pts);
    }
    if (backward) {
        Backward &b = p.bw;
        p.Bsum = c.take<float>((size_t)p.T * p.NBR * N);
        b.Fout = c.take<float>(3 * (size_t)N);
        b.Zout = c.take<float>(9 * (size_t)N);
        b.energy = c.take<double>(1);
        b.virial = c.take<double>(9);
        b.pol = c.take<double>(3);
        b.terms = c.take<double>(8);
        b.Xvec = c.take<float>((size_t)(3 * p.H + 1) * N);
        b.delta = c.take<float>((size_t)p.H * N);
        b.Gam = c.take<float>((size_t)p.ndes * N);
        b.Gc = c.take<float>((size_t)p.T * p.NA * p.NBA * N);
        b.sums = c.take<double>(16);
        b.sW0 = c.take<double>((size_t)p.T * p.H * p.ndes);
        b.sVec = c.take<double>((size_t)p.T * (3 * p.H + 1));
        b.sCR = c.take<double>((size_t)p.T * p.NR * p.T * p.NBR);
        b.sCA = c.take<double>((size_t)p.T * p.T * p.NA * p.NBA);
        const int64_t widest = std::max(std::max<int64_t>((int64_t)p.H * p.ndes, 3 * p.H + 1),
                                        std::max<int64_t>((int64_t)p.NR * p.T * p.NBR, (int64_t)p.T * p.NA * p.NBA));
        b.partials = c.take<double>((size_t)((N + 1023) / 1024) * p.T * widest);
    }
    *bytes = (c.off + ALIGN - 1) / ALIGN * ALIGN;
    return QNEP_OK;
}

// the forward launch sequence shared by qnep_compute and qnep_backward
hipError_t run_forward(Plan &p) {
    hipError_t e;
#define FW_TRY(x)                        \
    do {                                 \
        e = (x);                         \
        if (e != hipSuccess) return e;   \
    } while (0)
    FW_TRY(fill_zero(p.flags, sizeof(int32_t) * 16, p.stream));
    FW_TRY(fill_zero(p.scalars, sizeof(double) * 64, p.stream));
    if (p.N == 0) return launch_zero_outputs(p);
    FW_TRY(launch_neighbors(p));
    FW_TRY(launch_descriptors(p));
    stage_mark(p, ST_DESC);
    FW_TRY(launch_mlp(p));
    FW_TRY(launch_charges(p));
    stage_mark(p, ST_MLP, 3);
    FW_TRY(launch_real_space(p));
    stage_mark(p, ST_REAL, 2);
    if (p.method == 0) {
        FW_TRY(launch_ewald(p));
    } else {
        FW_TRY(launch_pppm(p));
    }
    FW_TRY(launch_phi_mean(p));
    stage_mark(p, ST_PHI, 3);
    FW_TRY(launch_forces(p));
    FW_TRY(launch_finalize(p));
    stage_mark(p, ST_FINAL, 1);
#undef FW_TRY
    return hipSuccess;
}

qnep_status check_model(const qnep_hparams *hp, int prec) {
    if (!hp) return fail(QNEP_E_INVALID_ARG, "null hyper-parameters");
    if (hp->n_types < 1 || hp->n_types > MAX_T) return fail(QNEP_E_UNSUPPORTED, "n_types must be 1..4");
    if (hp->n_neu < 1 || hp->n_neu > MAX_NEU) return fail(QNEP_E_UNSUPPORTED, "n_neu must be 1..64");
    if (!(hp->rc_R > 0) || !(hp->rc_A > 0) || hp->rc_A > hp->rc_R)
        return fail(QNEP_E_INVALID_ARG, "cutoffs must satisfy 0 < rc_A <= rc_R");
    if (!nep_supported(hp->n_types, hp->n_max_R + 1, hp->n_max_A + 1, hp->basis_R + 1, hp->basis_A + 1, hp->l_max))
        return fail(QNEP_E_UNSUPPORTED,
                    "compiled descriptor sets: l_max = 4, basis 8, (n_max_R, n_max_A) = (4, 4) or (8, 6)");
    int ndes = (hp->n_max_R + 1) + (hp->n_max_A + 1) * hp->l_max;
    if (prec == QNEP_MLP_BF16 || prec == QNEP_MLP_BF16X3) {
        if (!mlp_bf16_supported(ndes, hp->n_neu)) return fail(QNEP_E_UNSUPPORTED, "BF16 MLP not available");
    } else if (prec != QNEP_MLP_FP32) {
        return fail(QNEP_E_INVALID_ARG, "mlp_precision must be QNEP_MLP_FP32, QNEP_MLP_BF16 or QNEP_MLP_BF16X3");
    }
    return QNEP_OK;
}

#define HIP_TRY(x)                                                                         \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess) return fail(QNEP_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

}  // namespace

extern "C" {

int64_t qnep_param_count(const qnep_hparams *hp) {
    if (!hp || hp->n_types < 1 || hp->n_neu < 1 || hp->n_max_R < 0 || hp->n_max_A < 0 || hp->l_max < 1)
        return -1;
    return param_count(*hp);
}

qnep_status qnep_model_create(const qnep_hparams *hp, int32_t mlp_precision, void **model) {
    if (!model) return fail(QNEP_E_INVALID_ARG, "null model pointer");
    qnep_status s = check_model(hp, mlp_precision);
    if (s != QNEP_OK) return s;
    Model *m = new Model();
    m->hp = *hp;
    m->prec = mlp_precision;
    m->cap_factor = 1.6;
    *model = m;
    return QNEP_OK;
}

qnep_status qnep_model_destroy(void *model) {
    Model *m = static_cast<Model *>(model);
    if (m) m->timer.destroy();
    delete m;
    return QNEP_OK;
}

qnep_status qnep_model_enable_timing(void *model, int32_t enable) {
    if (!model) return fail(QNEP_E_INVALID_ARG, "null model");
    Model *m = static_cast<Model *>(model);
    if (enable) HIP_TRY(m->timer.create());
    m->timer.on = enable != 0;
    return QNEP_OK;
}

qnep_status qnep_model_read_timing(void *model, double *ms, int64_t *launches, int32_t *calls) {
    if (!model) return fail(QNEP_E_INVALID_ARG, "null model");
    Timer &t = static_cast<Model *>(model)->timer;
    while (t.count > 0) HIP_TRY(t.drain_one());
    for (int k = 0; k < QNEP_N_STAGES; ++k) {
        if (ms) ms[k] = t.total[k];
        if (launches) launches[k] = t.launches[k];
        t.total[k] = 0.0;
        t.launches[k] = 0;
    }
    if (calls) *calls = t.calls;
    t.calls = 0;
    t.cur = -1;
    return QNEP_OK;
}

const char *qnep_stage_name(int32_t stage) {
    if (stage < 0 || stage >= QNEP_N_STAGES) return "invalid";
    return kStageNames[stage];
}

qnep_status qnep_model_set_capacity_factor(void *model, double factor) {
    if (!model || !(factor >= 1.0) || factor > 100.0) return fail(QNEP_E_INVALID_ARG, "factor must be in [1, 100]");
    static_cast<Model *>(model)->cap_factor = factor;
    return QNEP_OK;
}

qnep_status qnep_workspace_size(const void *model, const qnep_es_params *es, const qnep_system *sys,
                                size_t *bytes) {
    if (!model || !bytes) return fail(QNEP_E_INVALID_ARG, "null argument");
    Plan p;
    return make_plan(*static_cast<const Model *>(model), es, sys, nullptr, p, bytes);
}

qnep_status qnep_compute(void *model, const float *theta, const qnep_es_params *es, const qnep_system *sys,
                         const qnep_outputs *out, void *ws, size_t ws_bytes, void *stream) {
    if (!model || !theta || !out || !ws) return fail(QNEP_E_INVALID_ARG, "null argument");
    const Model &m = *static_cast<const Model *>(model);
    Plan p;
    size_t need = 0;
    qnep_status s = make_plan(m, es, sys, static_cast<char *>(ws), p, &need);
    if (s != QNEP_OK) return s;
    if (ws_bytes < need) return fail(QNEP_E_WORKSPACE, "workspace smaller than qnep_workspace_size()");
    if (p.N > 0 && (!sys->pos || !sys->type)) return fail(QNEP_E_INVALID_ARG, "null positions or types");
    p.pos = sys->pos;
    p.type = sys->type;
    p.theta = theta;
    p.out = *out;
    p.stream = static_cast<hipStream_t>(stream);
    Model &mm = *static_cast<Model *>(model);
    if (mm.timer.on) {
        p.timer = &mm.timer;
        HIP_TRY(mm.timer.begin(p.stream));
    }
    HIP_TRY(run_forward(p));
    return QNEP_OK;
}

qnep_status qnep_backward_workspace_size(const void *model, const qnep_es_params *es, const qnep_system *sys,
                                         size_t *bytes) {
    if (!model || !bytes) return fail(QNEP_E_INVALID_ARG, "null argument");
    Plan p;
    return make_plan(*static_cast<const Model *>(model), es, sys, nullptr, p, bytes, true);
}

qnep_status qnep_backward(void *model, const float *theta, const qnep_es_params *es, const qnep_system *sys,
                          double gE, const double *gP, float *d_pos, double *d_cell, float *d_theta, void *ws,
                          size_t ws_bytes, void *stream) {
    if (!model || !theta || !ws) return fail(QNEP_E_INVALID_ARG, "null argument");
    const Model &m = *static_cast<const Model *>(model);
    Plan p;
    size_t need = 0;
    qnep_status s = make_plan(m, es, sys, static_cast<char *>(ws), p, &need, true);
    if (s != QNEP_OK) return s;
    if (ws_bytes < need) return fail(QNEP_E_WORKSPACE, "workspace smaller than qnep_backward_workspace_size()");
    if (p.N == 0) return fail(QNEP_E_INVALID_ARG, "backward needs at least one atom");
    if (!sys->pos || !sys->type) return fail(QNEP_E_INVALID_ARG, "null positions or types");
    p.pos = sys->pos;
    p.type = sys->type;
    p.theta = theta;
    p.stream = static_cast<hipStream_t>(stream);
    Backward &b = p.bw;
    b.gE = gE;
    for (int a = 0; a < 3; ++a) b.gP[a] = gP ? gP[a] : 0.0;
    b.dpos = d_pos;
    b.dcell = d_cell;
    b.dtheta = d_theta;
    p.out = qnep_outputs{b.energy, b.Fout, b.virial, nullptr, nullptr, b.Zout, b.pol, b.terms};
    HIP_TRY(run_forward(p));
    HIP_TRY(launch_backward(p));
    return QNEP_OK;
}

qnep_status qnep_check_status(const void *ws, void *stream, int32_t *flags) {
    if (!ws || !flags) return fail(QNEP_E_INVALID_ARG, "null argument");
    HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    HIP_TRY(hipMemcpy(flags, ws, sizeof(int32_t), hipMemcpyDeviceToHost));
    return QNEP_OK;
}

const char *qnep_status_string(qnep_status s) {
    switch (s) {
        case QNEP_OK: return "ok";
        case QNEP_E_INVALID_ARG: return "invalid argument";
        case QNEP_E_UNSUPPORTED: return "unsupported configuration";
        case QNEP_E_WORKSPACE: return "workspace too small";
        case QNEP_E_DEVICE: return "device error";
        case QNEP_E_INTERNAL: return "internal error";
        case QNEP_E_CAPACITY: return "device capacity exceeded";
    }
    return "unknown status";
}

const char *qnep_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
