// C ABI of libqnep (declared in include/qnep.h): validation, workspace layout and
// the launch sequence of one qNEP evaluation on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "batch.h"
#include "plan.h"

namespace qnep {
hipError_t snes_sample(int64_t d, int C, const float *mu, const float *sigma, const float *noise, float *thetas,
                       hipStream_t st);
hipError_t snes_update(int64_t d, int C, const double *loss, const float *noise, double eta_mu, double eta_sigma,
                       float *mu, float *sigma, hipStream_t st);
bool nep_supported(int T, int NR, int NA, int NBR, int NBA, int LMAX);
hipError_t md_kick_drift(const Plan &p, const double *masses, double dt, float *pos, float *vel, const float *F);
hipError_t md_kick_record(const Plan &p, const double *masses, double dt, float *vel, const float *F,
                          const float *Z, const double *energy, const double *pol, double *sums, double *row);
hipError_t launch_phi_mean(const Plan &p);
bool mlp_bf16_supported(int ndes, int H);
int masked_outer_chunks(int N);  // atom chunks of the reverse pass's parameter sums
int radial_record_floats(int NB);
int reduce_tmp_doubles();
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
    "radial_forces", "angular_forces", "assemble", "finalize", "other"};

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
    BatchPlan batch;
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
    const int np = (sys->pbc[0] != 0) + (sys->pbc[1] != 0) + (sys->pbc[2] != 0);
    if (np != 0 && np != 3) return fail(QNEP_E_UNSUPPORTED, "pbc must be {1,1,1} or {0,0,0}");
    p.iso = np == 0 ? 1 : 0;
    if (p.iso) {
        if (es->method != QNEP_ES_DIRECT)
            return fail(QNEP_E_INVALID_ARG, "an isolated system (pbc = 0) takes method QNEP_ES_DIRECT");
    } else {
        if (es->mode != 1 && es->mode != 2) return fail(QNEP_E_INVALID_ARG, "mode must be 1 or 2");
        if (es->method != 0 && es->method != 1)
            return fail(QNEP_E_INVALID_ARG, "a periodic system takes method 0 (Ewald) or 1 (PPPM)");
        if (!(es->alpha > 0)) return fail(QNEP_E_INVALID_ARG, "alpha must be positive");
        if (es->mode == 1 && !(es->rc_coul > 0)) return fail(QNEP_E_INVALID_ARG, "rc_coul must be positive");
    }
    p.mode = p.iso ? 1 : es->mode;
    p.method = es->method;
    p.alpha = es->alpha;
    p.rc_coul = es->rc_coul;
    p.kmax = es->kmax;
    p.kinc = es->kmax_inclusive ? 1 : 0;
    p.order = es->order;
    p.qtot = es->q_total;
    for (int a = 0; a < 3; ++a) {
        if (!std::isfinite(es->efield[a])) return fail(QNEP_E_INVALID_ARG, "efield must be finite");
        p.efield[a] = (float)es->efield[a];
    }
    for (int a = 0; a < 3; ++a) p.mesh[a] = es->mesh[a];
    std::memcpy(p.cell.h, sys->cell, sizeof(double) * 9);
    if (!invert_cell(p.cell.h, p.cell.hinv, &p.vol))
        return fail(QNEP_E_INVALID_ARG, "cell must be non-singular and right-handed");
    double w[3];
    cell_widths(p.cell.h, p.vol, w);
    // bins of about rc_R / 2 across rows and rc_R / 4 along c: a stencil row (one atom
    // range per image) is trimmed to the cutoff sphere in steps of a quarter cutoff
    const double rbin = 0.5 * std::max(p.rcR, p.rcA);
    for (int a = 0; a < 3; ++a) {
        p.nc[a] = std::max(1, (int)std::floor(w[a] / (a == 2 ? 0.5 * rbin : rbin)));
        p.mR[a] = (int)std::ceil(std::max(p.rcR, p.rcA) * p.nc[a] / w[a] - 1e-12);
        p.mC[a] = p.iso ? 1 : (int)std::ceil(p.rc_coul * p.nc[a] / w[a] - 1e-12);
        if (p.mR[a] < 1) p.mR[a] = 1;
        if (p.mC[a] < 1) p.mC[a] = 1;
        if (p.mR[a] > 3 * p.nc[a] || (p.mode == 1 && p.mC[a] > 3 * p.nc[a]))
            return fail(QNEP_E_UNSUPPORTED, "cell thinner than a third of a cutoff along an axis");
    }
    p.ncell = p.nc[0] * p.nc[1] * p.nc[2];
    // an isolated system's box is mostly empty: its mean density says nothing about the
    // local one, so a condensed-matter density (0.15 per cubic Angstrom) is assumed, and
    // no atom can have more than N - 1 neighbours
    const double density = p.iso ? std::max(p.N / p.vol, 0.15) : p.N / p.vol;
    p.capR = capacity(density, p.rcR, m.cap_factor);
    p.capA = capacity(density, p.rcA, m.cap_factor);
    if (p.iso) {  // capacities stay multiples of 8 (rows are read in 16- and 32-byte pieces)
        p.capR = std::max(8, std::min(p.capR, (p.N + 7) / 8 * 8));
        p.capA = std::max(8, std::min(p.capA, (p.N + 7) / 8 * 8));
    }
    p.nblk = (p.N + RED_THREADS - 1) / RED_THREADS;
    int64_t red_blocks = std::max(p.nblk, 1);
    red_blocks = std::max<int64_t>(red_blocks, ((int64_t)p.N * PARTIALS_LANES_MAX + RED_THREADS - 1) / RED_THREADS);
    if (p.iso) {
        // the direct sum over all pairs: blocks of RED_THREADS atoms
    } else if (p.method == 0) {
        if (!(p.kmax > 0)) return fail(QNEP_E_INVALID_ARG, "kmax must be positive for Ewald");
        for (int a = 0; a < 3; ++a) {
            const double *v = p.cell.h + 3 * a;
            double len = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            p.nk_box[a] = (int)std::floor(p.kmax * len / (2.0 * M_PI)) + 1;
        }
        int64_t nh = count_half_k(p.cell.hinv, p.nk_box[0], p.nk_box[1], p.nk_box[2], p.kmax, p.kinc);
        p.nk_cap = nh + 16;
        p.row_cap = (2 * p.nk_box[0] + 1) * (2 * p.nk_box[1] + 1);
        p.NZP = (p.nk_box[2] + 1 + 15) / 16 * 16;
        p.NZ4 = (p.nk_box[2] + 1 + 1) / 2 * 2;
        if (ewald_atoms_lds_bytes(p.NZ4) > 65536)
            return fail(QNEP_E_UNSUPPORTED, "Ewald: too many wave vectors along the third cell vector (kmax |c| / 2 pi > 93)");
        // about two thousand work-groups for each matrix-core product
        const int row_blocks = (p.row_cap + 63) / 64, zb = (p.NZP + 31) / 32;
        p.s_chunks = std::max(1, std::min((p.N + 63) / 64, 2048 / std::max(1, row_blocks * zb)));
        p.s_chunk = ((p.N + p.s_chunks - 1) / p.s_chunks + 1) / 2 * 2;
        const int atom_blocks = std::max(1, (p.N + 127) / 128);
        p.r_chunks = std::max(1, std::min((p.row_cap + 1) / 2, 2048 / atom_blocks));
        p.r_chunk = ((p.row_cap + p.r_chunks - 1) / p.r_chunks + 1) / 2 * 2;
        red_blocks = std::max<int64_t>(red_blocks, ((int64_t)p.row_cap * p.NZP + 255) / 256);
    } else {
        if (p.order != 5) return fail(QNEP_E_UNSUPPORTED, "PPPM assignment order must be 5");
        for (int a = 0; a < 3; ++a)
            if (!fft_length_supported(p.mesh[a]))
                return fail(QNEP_E_UNSUPPORTED, "mesh sizes must be products of 2, 3, 5 up to 1024");
        p.mesh_pts = (int64_t)p.mesh[0] * p.mesh[1] * p.mesh[2];
        red_blocks = std::max<int64_t>(red_blocks, (p.mesh_pts + 255) / 256);
        // the influence kernel: one work-group per row along c, at most 4096
        red_blocks = std::max<int64_t>(red_blocks, std::min<int64_t>((int64_t)p.mesh[0] * p.mesh[1], 4096));
        BrickGeom bg;
        p.bricks = spread_bricks(p.mesh, p.nc, &bg);
        for (int a = 0; a < 3; ++a) {
            p.brickP[a] = p.bricks ? bg.P[a] : 0;
            p.brickNb[a] = p.bricks ? bg.nb[a] : 0;
        }
    }
    p.partials_cap = red_blocks * 11;
    const int64_t N = std::max(p.N, 1);
    Carver c{base, 0, base == nullptr};
    p.flags = c.take<int32_t>(16);
    p.scalars = c.take<double>(64);
    p.partials = c.take<double>(p.partials_cap);
    p.red_tmp = c.take<double>(reduce_tmp_doubles());
    p.cid = c.take<int>(N);
    p.cell_count = c.take<int>(p.ncell);
    p.cell_start = c.take<int>(p.ncell + 1);
    p.cell_cursor = c.take<int>(p.ncell);
    p.scan_tmp = c.take<int>((p.ncell + 1023) / 1024 + 1);
    p.perm = c.take<int>(N);
    p.xyzt = c.take<float4>(N);
    p.xyzq = c.take<float4>(N);
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
    p.hT = c.take<float>((size_t)p.T * radial_record_floats(p.NBR) * N);
    p.pairFA = c.take<float>((size_t)8 * p.capA * N);
    p.Fnep = c.take<float>(3 * (size_t)N);
    p.Znep = c.take<float>(9 * (size_t)N);
    p.Vat = c.take<float>(6 * (size_t)N);
    p.Siso = c.take<float>(p.iso ? 3 * (size_t)N : 1);
    if (p.iso) {
    } else if (p.method == 0) {
        p.kvec = c.take<float4>(2 * (size_t)p.nk_cap);  // kv then kn (int4)
        p.kcount = c.take<int>(1);
        p.krows = c.take<int4>(p.row_cap);
        p.krowoff = c.take<int>(p.row_cap);
        p.knrows = c.take<int>(1);
        p.ewX = c.take<float2>((size_t)(2 * p.nk_box[0] + 1) * N);
        p.ewY = c.take<float2>((size_t)(2 * p.nk_box[1] + 1) * N);
        p.ewZ = c.take<float2>((size_t)p.NZP * N);
        p.Spart = c.take<float>((size_t)p.s_chunks * p.row_cap * p.NZP * 2);
        p.Ubox = c.take<float2>((size_t)p.row_cap * 4 * p.NZ4);
        p.ephi = c.take<float>((size_t)p.r_chunks * 4 * N);
        p.Sk = c.take<float2>(p.nk_cap);
    } else {
        if (!p.bricks) p.rho = c.take<float>(p.mesh_pts);
        p.meshA = c.take<float2>(p.mesh_pts);
        p.meshAB = c.take<float2>(2 * p.mesh_pts);
        p.meshV = c.take<float2>(3 * p.mesh_pts);
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
        b.partials = c.take<double>((size_t)masked_outer_chunks(N) * p.T * widest);
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
    if (p.iso) {
        FW_TRY(launch_direct_coulomb(p));
        FW_TRY(launch_centroid(p));
    } else {
        FW_TRY(launch_real_space(p));  // marks the real-space kernel itself
        stage_mark(p, ST_OTHER, 1);
        if (p.method == 0) {
            FW_TRY(launch_ewald(p));
        } else {
            FW_TRY(launch_pppm(p));
        }
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

// Sizes, per-structure records and workspace layout of a batch (dry run when base is null).
qnep_status batch_layout(const Model &m, const qnep_es_params *es, const qnep_batch *bt, int C_max, char *base,
                         BatchPlan &bp, size_t *bytes) {
    const qnep_hparams &hp = m.hp;
    if (!es || !bt || !bytes) return fail(QNEP_E_INVALID_ARG, "null argument");
    if (bt->n_structures < 1 || !bt->offsets || !bt->cells)
        return fail(QNEP_E_INVALID_ARG, "batch needs n_structures >= 1, offsets and cells");
    if (C_max < 1) return fail(QNEP_E_INVALID_ARG, "max_candidates must be >= 1");
    const int T = hp.n_types, NR = hp.n_max_R + 1, NA = hp.n_max_A + 1, NB = hp.basis_R + 1;
    if (hp.basis_A != hp.basis_R || hp.l_max != 4 || !batch_supported(T, NR, NA, NB))
        return fail(QNEP_E_UNSUPPORTED, "batched path: l_max = 4, basis_R = basis_A = 8, (n_max_R, n_max_A) = (4, 4) or (8, 6)");
    if (param_count(hp) > BATCH_MAX_THETA) return fail(QNEP_E_UNSUPPORTED, "batched path: more than 12288 parameters");
    if (es->method != 0) return fail(QNEP_E_UNSUPPORTED, "batched path: Ewald only (method 0)");
    if (es->mode != 1 && es->mode != 2) return fail(QNEP_E_INVALID_ARG, "mode must be 1 or 2");
    if (!(es->alpha > 0) || !(es->kmax > 0)) return fail(QNEP_E_INVALID_ARG, "alpha and kmax must be positive");
    if (es->mode == 1 && !(es->rc_coul > 0)) return fail(QNEP_E_INVALID_ARG, "rc_coul must be positive");
    const int S = bt->n_structures;
    if (bt->offsets[0] != 0) return fail(QNEP_E_INVALID_ARG, "offsets[0] must be 0");
    bp = BatchPlan{};
    bp.S = S;
    bp.C_max = C_max;
    bp.ncomp = (bt->flags & QNEP_BATCH_VIRIAL) ? BATCH_COMP_VIRIAL : BATCH_COMP_FORCE;
    bp.qtot = es->q_total;
    bp.st.resize(S);
    double max_density = 0.0;
    int64_t mat = 0, k0 = 0, ph0 = 0, tile0 = 0;
    for (int s = 0; s < S; ++s) {
        const int64_t n = bt->offsets[s + 1] - bt->offsets[s];
        if (n < 1 || n > BATCH_MAX_ATOMS) return fail(QNEP_E_UNSUPPORTED, "batched path: 1..2048 atoms per structure");
        BatchStruct &b = bp.st[s];
        std::memcpy(b.h, bt->cells + 9 * s, sizeof(double) * 9);
        if (!invert_cell(b.h, b.hinv, &b.vol)) return fail(QNEP_E_INVALID_ARG, "cell must be non-singular and right-handed");
        double w[3];
        cell_widths(b.h, b.vol, w);
        b.atom0 = bt->offsets[s];
        b.n = (int)n;
        for (int a = 0; a < 3; ++a) {
            b.mR[a] = (int)std::floor(std::max(hp.rc_R, hp.rc_A) / w[a] + 0.5) + 1;
            b.mC[a] = es->mode == 1 ? (int)std::floor(es->rc_coul / w[a] + 0.5) + 1 : 0;
            if (b.mR[a] > 8 || b.mC[a] > 8) return fail(QNEP_E_UNSUPPORTED, "batched path: cell thinner than an eighth of a cutoff");
            const double *v = b.h + 3 * a;
            b.kbox[a] = (int)std::floor(es->kmax * std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / (2.0 * M_PI)) + 1;
        }
        b.kcap = (int)count_half_k(b.hinv, b.kbox[0], b.kbox[1], b.kbox[2], es->kmax, es->kmax_inclusive);
        b.mat0 = mat;
        b.k0 = k0;
        b.ph0 = ph0;
        b.tile0 = tile0;
        b.group = batch_class(b.n);
        mat += (int64_t)bp.ncomp * n * n;
        k0 += b.kcap;
        ph0 += (int64_t)b.kcap * n;
        tile0 += (int64_t)((n + 15) / 16) * ((n + 15) / 16);
        max_density = std::max(max_density, n / b.vol);
        bp.max_atoms = std::max(bp.max_atoms, (int)n);
    }
    bp.n_total = bt->offsets[S];
    bp.mat_total = mat;
    bp.k_total = k0;
    bp.ph_total = ph0;
    bp.n_tiles = tile0;
    bp.capR = capacity(max_density, hp.rc_R, m.cap_factor);
    const int ndes = NR + 4 * NA;
    bp.per_slot = (int64_t)(3 * ndes + LM * NA) * bp.max_atoms;
    // queue order: size classes from large to small, larger structures first inside a class
    bp.order.resize(S);
    for (int s = 0; s < S; ++s) bp.order[s] = s;
    std::stable_sort(bp.order.begin(), bp.order.end(), [&](int x, int y) { return bp.st[x].n > bp.st[y].n; });
    for (int k = 0; k < BATCH_CLASSES; ++k) {
        bp.cls_lo[k] = S;
        bp.cls_hi[k] = 0;
    }
    for (int r = 0; r < S; ++r) {
        const int k = bp.st[bp.order[r]].group;
        bp.cls_lo[k] = std::min(bp.cls_lo[k], r);
        bp.cls_hi[k] = std::max(bp.cls_hi[k], r + 1);
    }
    Carver c{base, 0, base == nullptr};
    bp.flags = c.take<int32_t>(16);
    bp.counter = c.take<int>(16);
    bp.st_d = c.take<BatchStruct>(S);
    bp.order_d = c.take<int>(S);
    bp.ts = c.take<int>(bp.n_total);
    bp.cntR = c.take<int>(bp.n_total);
    bp.cntA = c.take<int>(bp.n_total);
    bp.list = c.take<float4>((size_t)bp.n_total * bp.capR);
    bp.kv = c.take<float4>(bp.k_total);
    bp.kcount = c.take<int>(S);
    bp.ph = c.take<float2>(bp.ph_total);
    bp.mats = c.take<float>(bp.mat_total);
    bp.stats = c.take<double>((size_t)S * C_max * 4);
    bp.rmse = c.take<double>((size_t)C_max * 4);
    bp.scratch = c.take<float>((size_t)BATCH_MAX_SLOTS * bp.per_slot);
    bp.F = LM * NA + 2 * ndes;
    bp.C16_max = (C_max + 15) / 16 * 16;
    bp.persist = c.take<float>((size_t)bp.F * C_max * bp.n_total);
    bp.qbuf = c.take<float>((size_t)bp.n_total * bp.C16_max);
    bp.ybuf = c.take<float>((size_t)bp.ncomp * C_max * bp.n_total);
    bp.iscal = c.take<double>((size_t)S * C_max * 2);
    bp.grad = (bt->flags & QNEP_BATCH_GRADIENT) != 0;
    if (bp.grad) {
        bp.per_slot_adj = batch_adj_floats(T, NR, NA, NB, hp.n_neu) * bp.max_atoms;
        bp.fbuf = c.take<float>((size_t)C_max * 3 * bp.n_total);
        bp.grow = c.take<float>((size_t)S * C_max * param_count(hp));
        bp.adj_scratch = c.take<float>((size_t)BATCH_ADJ_SLOTS * bp.per_slot_adj);
    }
    bp.need = (c.off + ALIGN - 1) / ALIGN * ALIGN;
    *bytes = bp.need;
    return QNEP_OK;
}

#define HIP_TRY(x)                                                                         \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess) return fail(QNEP_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

// workspace of qnep_compute_static (see the header for its size and sharing rules)
__device__ __align__(256) char scratch[QNEP_STATIC_WORKSPACE_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
char *g_scratch_ptr[MAX_DEVICES] = {};

// device address of this GPU's `scratch`, resolved once per device with that device current
qnep_status static_workspace(char **ptr) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(QNEP_E_UNSUPPORTED, "device ordinal beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *addr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch)));
        if (!addr) return fail(QNEP_E_DEVICE, "hipGetSymbolAddress returned a null address");
        g_scratch_ptr[dev] = static_cast<char *>(addr);
    }
    *ptr = g_scratch_ptr[dev];
    return QNEP_OK;
}

__global__ void k_copy_flags(const int32_t *__restrict__ src, int32_t *__restrict__ dst) {
    if (threadIdx.x == 0) dst[0] = src[0];
}

hipError_t copy_flags(const int32_t *src, int32_t *dst, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_flags, dim3(1), dim3(64), 0, st, src, dst);
    return hipGetLastError();
}

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

// The allocation-free variant of qnep_compute: the whole workspace lives in `scratch`,
// a file-scope device array (one per GPU, held while the process runs).  Host code
// never passes the array's name to a kernel or a copy: its device address is resolved
// with hipGetSymbolAddress once per device (the first call on that device) and only
// that address is used afterwards.
qnep_status qnep_compute_static(void *model, const float *theta, const qnep_es_params *es, const qnep_system *sys,
                                const qnep_outputs *out, int32_t *flags_out, void *stream) {
    if (!model || !theta || !out) return fail(QNEP_E_INVALID_ARG, "null argument");
    const Model &m = *static_cast<const Model *>(model);
    Plan p;
    size_t need = 0;
    qnep_status s = make_plan(m, es, sys, nullptr, p, &need);
    if (s != QNEP_OK) return s;
    if (need > (size_t)QNEP_STATIC_WORKSPACE_BYTES)
        return fail(QNEP_E_WORKSPACE, "structure needs " + std::to_string(need) +
                                          " bytes of workspace; the static workspace holds " +
                                          std::to_string((size_t)QNEP_STATIC_WORKSPACE_BYTES));
    if (p.N > 0 && (!sys->pos || !sys->type)) return fail(QNEP_E_INVALID_ARG, "null positions or types");
    char *ws = nullptr;
    s = static_workspace(&ws);
    if (s != QNEP_OK) return s;
    s = make_plan(m, es, sys, ws, p, &need);
    if (s != QNEP_OK) return s;
    p.pos = sys->pos;
    p.type = sys->type;
    p.theta = theta;
    p.out = *out;
    p.stream = static_cast<hipStream_t>(stream);
    p.timer = nullptr;  // no event records: nothing but kernel launches is enqueued
    HIP_TRY(run_forward(p));
    if (flags_out) HIP_TRY(copy_flags(p.flags, flags_out, p.stream));
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
    if (p.efield[0] != 0.f || p.efield[1] != 0.f || p.efield[2] != 0.f)
        return fail(QNEP_E_UNSUPPORTED, "the adjoint is of the field-free energy: pass efield = 0");
    if (p.N == 0) return fail(QNEP_E_INVALID_ARG, "backward needs at least one atom");
    if (!sys->pos || !sys->type) return fail(QNEP_E_INVALID_ARG, "null positions or types");
    p.pos = sys->pos;
    p.type = sys->type;
    p.theta = theta;
    p.stream = static_cast<hipStream_t>(stream);
    Backward &b = p.bw;
    b.gE = gE;
    for (int a = 0; a < 3; ++a) b.gP[a] = gP ? gP[a] : 0.0;
    if (d_cell && (b.gP[0] != 0.0 || b.gP[1] != 0.0 || b.gP[2] != 0.0))
        return fail(QNEP_E_UNSUPPORTED,
                    "d_cell covers the energy term only: pass gP = 0 (or NULL) when d_cell is requested");
    b.dpos = d_pos;
    b.dcell = d_cell;
    b.dtheta = d_theta;
    p.out = qnep_outputs{b.energy, b.Fout, b.virial, nullptr, nullptr, b.Zout, b.pol, b.terms};
    HIP_TRY(run_forward(p));
    HIP_TRY(launch_backward(p));
    return QNEP_OK;
}

namespace {
// device buffers of the MD driver, after the evaluation's workspace
struct MdBuffers {
    float *F = nullptr, *Z = nullptr;
    double *energy = nullptr, *pol = nullptr, *sums = nullptr;
};

qnep_status md_layout(const Model &m, const qnep_es_params *es, int64_t n_atoms, const double *cell, char *ws,
                      Plan &p, MdBuffers &b, size_t *bytes) {
    if (!cell) return fail(QNEP_E_INVALID_ARG, "null cell");
    qnep_system sys{n_atoms, nullptr, nullptr, {0}, {1, 1, 1}};
    std::memcpy(sys.cell, cell, sizeof(double) * 9);
    size_t need = 0;
    qnep_status s = make_plan(m, es, &sys, ws, p, &need);
    if (s != QNEP_OK) return s;
    Carver c{ws, need, ws == nullptr};
    const size_t N = (size_t)std::max<int64_t>(n_atoms, 1);
    b.F = c.take<float>(3 * N);
    b.Z = c.take<float>(9 * N);
    b.energy = c.take<double>(1);
    b.pol = c.take<double>(3);
    b.sums = c.take<double>(4);
    *bytes = (c.off + ALIGN - 1) / ALIGN * ALIGN;
    return QNEP_OK;
}
}  // namespace

qnep_status qnep_md_workspace_size(const void *model, const qnep_es_params *es, int64_t n_atoms,
                                   const double *cell, size_t *bytes) {
    if (!model || !bytes) return fail(QNEP_E_INVALID_ARG, "null argument");
    Plan p;
    MdBuffers b;
    return md_layout(*static_cast<const Model *>(model), es, n_atoms, cell, nullptr, p, b, bytes);
}

qnep_status qnep_md_nve(void *model, const float *theta, const qnep_es_params *es, const qnep_md_params *md,
                        int64_t n_atoms, const int32_t *type, const double *cell, float *pos, float *vel,
                        double *series, void *ws, size_t ws_bytes, void *stream) {
    if (!model || !theta || !md || !pos || !vel || !type || !series || !ws)
        return fail(QNEP_E_INVALID_ARG, "null argument");
    if (n_atoms < 1) return fail(QNEP_E_INVALID_ARG, "MD needs at least one atom");
    if (!(md->dt > 0) || !std::isfinite(md->dt) || md->n_steps < 0)
        return fail(QNEP_E_INVALID_ARG, "dt must be positive and n_steps non-negative");
    const Model &m = *static_cast<const Model *>(model);
    if (!md->masses) return fail(QNEP_E_INVALID_ARG, "null masses");
    for (int t = 0; t < m.hp.n_types; ++t)
        if (!(md->masses[t] > 0) || !std::isfinite(md->masses[t]))
            return fail(QNEP_E_INVALID_ARG, "masses must be positive");
    Plan p;
    MdBuffers b;
    size_t need = 0;
    qnep_status s = md_layout(m, es, n_atoms, cell, static_cast<char *>(ws), p, b, &need);
    if (s != QNEP_OK) return s;
    if (ws_bytes < need) return fail(QNEP_E_WORKSPACE, "workspace smaller than qnep_md_workspace_size()");
    p.pos = pos;
    p.type = type;
    p.theta = theta;
    p.stream = static_cast<hipStream_t>(stream);
    p.out = qnep_outputs{b.energy, b.F, nullptr, nullptr, nullptr, b.Z, b.pol, nullptr, nullptr};
    HIP_TRY(run_forward(p));
    HIP_TRY(md_kick_record(p, md->masses, 0.0, vel, b.F, b.Z, b.energy, b.pol, b.sums, series));
    for (int step = 1; step <= md->n_steps; ++step) {
        HIP_TRY(md_kick_drift(p, md->masses, md->dt, pos, vel, b.F));
        HIP_TRY(run_forward(p));
        HIP_TRY(md_kick_record(p, md->masses, md->dt, vel, b.F, b.Z, b.energy, b.pol, b.sums,
                               series + (size_t)8 * step));
    }
    return QNEP_OK;
}

qnep_status qnep_check_status(const void *ws, void *stream, int32_t *flags) {
    if (!ws || !flags) return fail(QNEP_E_INVALID_ARG, "null argument");
    HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    HIP_TRY(hipMemcpy(flags, ws, sizeof(int32_t), hipMemcpyDeviceToHost));
    return QNEP_OK;
}

qnep_status qnep_batch_workspace_size(const void *model, const qnep_es_params *es, const qnep_batch *batch,
                                      int32_t max_candidates, size_t *bytes) {
    if (!model) return fail(QNEP_E_INVALID_ARG, "null model");
    BatchPlan bp;
    return batch_layout(*static_cast<const Model *>(model), es, batch, max_candidates, nullptr, bp, bytes);
}

qnep_status qnep_batch_prepare(void *model, const qnep_es_params *es, const qnep_batch *batch,
                               int32_t max_candidates, void *ws, size_t ws_bytes, void *stream) {
    if (!model || !ws) return fail(QNEP_E_INVALID_ARG, "null argument");
    Model &m = *static_cast<Model *>(model);
    BatchPlan bp;
    size_t need = 0;
    qnep_status s = batch_layout(m, es, batch, max_candidates, static_cast<char *>(ws), bp, &need);
    if (s != QNEP_OK) return s;
    if (ws_bytes < need) return fail(QNEP_E_WORKSPACE, "workspace smaller than qnep_batch_workspace_size()");
    if (!batch->pos || !batch->type) return fail(QNEP_E_INVALID_ARG, "null positions or types");
    if (es->efield[0] != 0.0 || es->efield[1] != 0.0 || es->efield[2] != 0.0)
        return fail(QNEP_E_UNSUPPORTED, "batched evaluation has no external field: pass efield = 0");
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    bp.cus = cus > 0 ? cus : 256;
    // keep the tuned choices of an earlier prepare
    if (m.batch.ready) {
        for (int k = 0; k < BATCH_CLASSES; ++k) bp.groups[k] = m.batch.groups[k];
        bp.slots_per_cu = m.batch.slots_per_cu;
    }
    m.batch = std::move(bp);
    BatchPlan &b = m.batch;
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(fill_zero(b.flags, sizeof(int32_t) * 16, st));
    HIP_TRY(hipMemcpyAsync(b.st_d, b.st.data(), sizeof(BatchStruct) * b.S, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(b.order_d, b.order.data(), sizeof(int) * b.S, hipMemcpyHostToDevice, st));
    const qnep_hparams &hp = m.hp;
    HIP_TRY(batch_setup(b.st_d, b.S, b.n_total, b.n_tiles, b.ph_total, batch->pos, batch->type, hp.n_types,
                        hp.rc_R, hp.rc_A, b.list, b.cntR, b.cntA, b.capR, b.ts, b.flags, *es, b.kv, b.kcount, b.ph,
                        b.ncomp, b.mats, st));
    b.ws = ws;
    b.ready = true;
    return QNEP_OK;
}

namespace {
qnep_status batch_args(const Model &m, const float *thetas, int C, const qnep_batch_targets *tg,
                       const qnep_batch_outputs *out, const void *ws, size_t ws_bytes, BatchArgs &a) {
    const BatchPlan &b = m.batch;
    if (!b.ready || ws != b.ws) return fail(QNEP_E_INVALID_ARG, "workspace was not prepared by qnep_batch_prepare");
    if (ws_bytes < b.need) return fail(QNEP_E_WORKSPACE, "workspace smaller than qnep_batch_workspace_size()");
    if (!thetas || !tg || !out || !tg->energy || !tg->forces || !out->losses)
        return fail(QNEP_E_INVALID_ARG, "null thetas, targets or losses");
    if (C < 1 || C > b.C_max) return fail(QNEP_E_INVALID_ARG, "n_candidates must be in [1, max_candidates]");
    if (out->virial && b.ncomp != BATCH_COMP_VIRIAL)
        return fail(QNEP_E_INVALID_ARG, "virial output needs QNEP_BATCH_VIRIAL at prepare");
    const qnep_hparams &hp = m.hp;
    const int T = hp.n_types, NR = hp.n_max_R + 1, NA = hp.n_max_A + 1, NB = hp.basis_R + 1;
    const int ndes = NR + 4 * NA;
    a = BatchArgs{};
    a.st = b.st_d;
    a.order = b.order_d;
    a.S = b.S;
    a.C = C;
    a.n_items = b.S * C;
    a.counter = b.counter;
    a.flags = b.flags;
    a.list = b.list;
    a.cntR = b.cntR;
    a.cntA = b.cntA;
    a.types = b.ts;
    a.capR = b.capR;
    a.mats = b.mats;
    a.ncomp = b.ncomp;
    a.thetas = thetas;
    a.off_cA = (int64_t)T * T * NR * NB;
    a.off_nn = a.off_cA + (int64_t)T * T * NA * NB;
    a.per_species = (int64_t)hp.n_neu * ndes + 3 * hp.n_neu + 1;
    a.off_b1E = a.off_nn + T * a.per_species;
    a.off_s = a.off_b1E + 1;
    a.n_theta = a.off_s + 1;
    a.H = hp.n_neu;
    a.ndes = ndes;
    a.prec = m.prec;
    a.rcR = hp.rc_R;
    a.rcA = hp.rc_A;
    a.qtot = b.qtot;
    a.E_ref = tg->energy;
    a.F_ref = tg->forces;
    a.n_total = b.n_total;
    a.losses = out->losses;
    a.energy = out->energy;
    a.virial = out->virial;
    a.forces = out->forces;
    a.charges = out->charges;
    a.stats = b.stats;
    a.scratch = b.scratch;
    a.max_atoms = b.max_atoms;
    a.persist = b.persist;
    a.F = b.F;
    a.qbuf = b.qbuf;
    a.C16 = (a.C + 15) / 16 * 16;
    a.ybuf = b.ybuf;
    a.iscal = b.iscal;
    return QNEP_OK;
}

hipError_t batch_run(const Model &m, const BatchArgs &a, int item_begin, int item_end, const int *groups,
                     int slots_per_cu, hipStream_t st) {
    const BatchPlan &b = m.batch;
    const qnep_hparams &hp = m.hp;
    hipError_t e = fill_zero(b.counter, sizeof(int) * 16, st);
    if (e != hipSuccess) return e;
    int slots = std::min(b.cus * slots_per_cu, BATCH_MAX_SLOTS);
    return batch_eval(a, hp.n_types, hp.n_max_R + 1, hp.n_max_A + 1, hp.basis_R + 1, slots, item_begin, item_end,
                      make_int4(groups[0], groups[1], groups[2], groups[3]), st);
}
}  // namespace

qnep_status qnep_batch_compute(void *model, const float *thetas, int32_t n_candidates,
                               const qnep_batch_targets *targets, const qnep_batch_outputs *outputs, void *ws,
                               size_t ws_bytes, void *stream) {
    if (!model) return fail(QNEP_E_INVALID_ARG, "null model");
    const Model &m = *static_cast<const Model *>(model);
    BatchArgs a;
    qnep_status s = batch_args(m, thetas, n_candidates, targets, outputs, ws, ws_bytes, a);
    if (s != QNEP_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(batch_run(m, a, 0, a.n_items, m.batch.groups, m.batch.slots_per_cu, st));
    if (outputs->loss) {
        const double lam[5] = {targets->lambda_e, targets->lambda_f, targets->lambda_q, targets->lambda_1,
                               targets->lambda_2};
        HIP_TRY(batch_loss(m.batch.stats, targets->energy, thetas, a.n_theta, a.S, a.C, a.qtot, lam, outputs->loss,
                           m.batch.rmse, st));
    }
    return QNEP_OK;
}

qnep_status qnep_snes_generation(void *model, float *mu, float *sigma, const float *noise, int32_t n_candidates,
                                 double eta_mu, double eta_sigma, const qnep_batch_targets *targets,
                                 const qnep_batch_outputs *outputs, float *thetas, void *ws, size_t ws_bytes,
                                 void *stream) {
    if (!model || !mu || !sigma || !noise || !thetas) return fail(QNEP_E_INVALID_ARG, "null argument");
    if (!outputs || !outputs->loss) return fail(QNEP_E_INVALID_ARG, "outputs->loss receives the fitness: required");
    if (n_candidates < 2 || n_candidates > 1024) return fail(QNEP_E_INVALID_ARG, "n_candidates must be in [2, 1024]");
    if (!(eta_mu > 0) || !std::isfinite(eta_mu)) return fail(QNEP_E_INVALID_ARG, "eta_mu must be positive");
    const Model &m = *static_cast<const Model *>(model);
    BatchArgs a;
    qnep_status s = batch_args(m, thetas, n_candidates, targets, outputs, ws, ws_bytes, a);
    if (s != QNEP_OK) return s;
    const int64_t d = a.n_theta;
    if (!(eta_sigma > 0)) eta_sigma = (3.0 + std::log((double)d)) / (5.0 * std::sqrt((double)d));
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_TRY(snes_sample(d, n_candidates, mu, sigma, noise, thetas, st));
    s = qnep_batch_compute(model, thetas, n_candidates, targets, outputs, ws, ws_bytes, stream);
    if (s != QNEP_OK) return s;
    HIP_TRY(snes_update(d, n_candidates, outputs->loss, noise, eta_mu, eta_sigma, mu, sigma, st));
    return QNEP_OK;
}

qnep_status qnep_batch_gradient(void *model, const float *thetas, int32_t n_candidates,
                                const qnep_batch_targets *targets, const qnep_batch_outputs *outputs,
                                float *d_thetas, void *ws, size_t ws_bytes, void *stream) {
    if (!model || !d_thetas) return fail(QNEP_E_INVALID_ARG, "null model or gradient");
    const Model &m = *static_cast<const Model *>(model);
    BatchArgs a;
    qnep_status s = batch_args(m, thetas, n_candidates, targets, outputs, ws, ws_bytes, a);
    if (s != QNEP_OK) return s;
    const BatchPlan &b = m.batch;
    if (!b.grad) return fail(QNEP_E_INVALID_ARG, "gradient needs QNEP_BATCH_GRADIENT at prepare");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const qnep_hparams &hp = m.hp;
    // forward (forces kept for the upstream force weights), then the aggregated loss
    float *F = outputs->forces ? outputs->forces : b.fbuf;
    a.forces = F;
    HIP_TRY(batch_run(m, a, 0, a.n_items, b.groups, b.slots_per_cu, st));
    const double lam[5] = {targets->lambda_e, targets->lambda_f, targets->lambda_q, targets->lambda_1,
                           targets->lambda_2};
    HIP_TRY(batch_loss(b.stats, targets->energy, thetas, a.n_theta, a.S, a.C, a.qtot, lam, outputs->loss, b.rmse, st));
    AdjArgs g{};
    g.forces = F;
    g.rmse = b.rmse;
    for (int k = 0; k < 5; ++k) g.lam[k] = lam[k];
    g.nf = 3.0 * (double)b.n_total;
    g.grow = b.grow;
    g.scratch = b.adj_scratch;
    HIP_TRY(fill_zero(b.counter, sizeof(int) * 16, st));
    const int slots = std::min(b.cus * 2, BATCH_ADJ_SLOTS);
    HIP_TRY(batch_adjoint(a, g, hp.n_types, hp.n_max_R + 1, hp.n_max_A + 1, hp.basis_R + 1, slots,
                          make_int4(b.groups[0], b.groups[1], b.groups[2], b.groups[3]), st));
    HIP_TRY(batch_grad_reduce(b.grow, thetas, a.n_theta, a.S, a.C, lam[3], lam[4], d_thetas, st));
    return QNEP_OK;
}

qnep_status qnep_batch_tune(void *model, const float *thetas, int32_t n_candidates,
                            const qnep_batch_targets *targets, const qnep_batch_outputs *outputs, void *ws,
                            size_t ws_bytes, void *stream, int32_t *choice) {
    if (!model) return fail(QNEP_E_INVALID_ARG, "null model");
    Model &m = *static_cast<Model *>(model);
    BatchArgs a;
    qnep_status s = batch_args(m, thetas, n_candidates, targets, outputs, ws, ws_bytes, a);
    if (s != QNEP_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(stream);
    BatchPlan &b = m.batch;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    // best of three timed runs (after one untimed run) of items [lo, hi)
    auto timed = [&](int lo, int hi, const int *groups, int spc, float *best) -> hipError_t {
        hipError_t e = batch_run(m, a, lo, hi, groups, spc, st);
        if (e != hipSuccess) return e;
        *best = 1e30f;
        for (int r = 0; r < 3; ++r) {
            if ((e = hipEventRecord(e0, st)) != hipSuccess) return e;
            if ((e = batch_run(m, a, lo, hi, groups, spc, st)) != hipSuccess) return e;
            if ((e = hipEventRecord(e1, st)) != hipSuccess) return e;
            if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
            float ms = 0.f;
            if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return e;
            *best = std::min(*best, ms);
        }
        return hipSuccess;
    };
    static const int lanes[] = {1, 2, 4, 8, 16};
    hipError_t err = hipSuccess;
    for (int k = 0; k < BATCH_CLASSES && err == hipSuccess; ++k) {
        if (b.cls_lo[k] >= b.cls_hi[k]) continue;
        float best = 1e30f;
        int pick = b.groups[k];
        for (int G : lanes) {
            int g[BATCH_CLASSES];
            for (int q = 0; q < BATCH_CLASSES; ++q) g[q] = b.groups[q];
            g[k] = G;
            float ms = 0.f;
            err = timed(b.cls_lo[k] * a.C, b.cls_hi[k] * a.C, g, b.slots_per_cu, &ms);
            if (err != hipSuccess) break;
            if (ms < best) {
                best = ms;
                pick = G;
            }
        }
        b.groups[k] = pick;
    }
    if (err == hipSuccess) {
        float best = 1e30f;
        int pick = b.slots_per_cu;
        for (int spc = 1; spc <= 4 && err == hipSuccess; ++spc) {
            float ms = 0.f;
            err = timed(0, a.n_items, b.groups, spc, &ms);
            if (err == hipSuccess && ms < best) {
                best = ms;
                pick = spc;
            }
        }
        b.slots_per_cu = pick;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fail(QNEP_E_DEVICE, std::string("batch tuning: ") + hipGetErrorString(err));
    if (choice) {
        for (int k = 0; k < BATCH_CLASSES; ++k) choice[k] = b.groups[k];
        choice[BATCH_CLASSES] = b.slots_per_cu;
    }
    // leave the outputs of the chosen configuration
    HIP_TRY(batch_run(m, a, 0, a.n_items, b.groups, b.slots_per_cu, st));
    if (outputs->loss) {
        const double lam[5] = {targets->lambda_e, targets->lambda_f, targets->lambda_q, targets->lambda_1,
                               targets->lambda_2};
        HIP_TRY(batch_loss(b.stats, targets->energy, thetas, a.n_theta, a.S, a.C, a.qtot, lam, outputs->loss, b.rmse, st));
    }
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
