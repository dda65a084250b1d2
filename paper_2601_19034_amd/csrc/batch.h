// Batched evaluation of many small periodic structures under many parameter vectors:
// the per-structure records and the argument block of the persistent launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/qnep.h"
#include "common.h"

namespace qnep {

constexpr int BATCH_THREADS = 256;
constexpr int BATCH_MAX_ATOMS = 2048;   // atoms per structure (LDS-resident per-atom state)
constexpr int BATCH_MAX_THETA = 12288;  // parameters staged in LDS per work item
constexpr int BATCH_COMP_FORCE = 4;     // pair matrices without the virial: A, G_x, G_y, G_z
constexpr int BATCH_COMP_VIRIAL = 10;   // ... and V_xx, V_yy, V_zz, V_xy, V_xz, V_yz

// One structure of the batch (host-built, copied to the workspace by the prepare call).
struct BatchStruct {
    double h[9], hinv[9];
    double vol;
    int64_t atom0;   // first atom in the packed caller arrays
    int64_t mat0;    // first float of its pair matrices [comp][j][i]
    int64_t k0;      // first entry of its half k-set
    int64_t ph0;     // first entry of its phase table [k][i]
    int64_t tile0;   // first 16 x 16 tile of the pair-matrix kernel
    int n;           // atoms
    int kcap;        // capacity of its half k-set (exact count)
    int mR[3];       // image range of the descriptor lists
    int mC[3];       // image range of the real-space Coulomb sum
    int kbox[3];     // integer box of the wave-vector enumeration
    int group;       // lanes per atom in the persistent kernel
};

// Argument block of the persistent kernel (passed by value).
struct BatchArgs {
    const BatchStruct *st;
    const int *order;        // structures, most expensive first
    int S, C, n_items;
    int *counter;            // work-queue head (zeroed before the launch)
    int32_t *flags;
    const float4 *list;      // [atom][capR] (dx, dy, dz, j | t_j << 24), angular pairs first
    const int *cntR, *cntA;
    const int *types;        // [n_total] species (validated copy)
    int capR;
    const float *mats;
    int ncomp;
    const float *thetas;     // [C][n_theta]
    int64_t n_theta, off_cA, off_nn, per_species, off_b1E, off_s;
    int H, ndes;
    int prec;                // network precision (QNEP_MLP_*)
    float rcR, rcA;
    double qtot;
    const double *E_ref;     // [S]
    const float *F_ref;      // [3][n_total]
    int64_t n_total;
    float *losses;           // [S][C][3]
    double *energy;          // [S][C]
    double *virial;          // [S][C][9]
    float *forces;           // [C][3][n_total]
    float *charges;          // [C][n_total]
    double *stats;           // [S][C][4]: E, sum |F - F_ref|^2, s sum q, 0
    float *scratch;          // per slot: [(3 ndes + 24 NA)][max_atoms]
    int max_atoms;
    // between the forward launches
    float *persist;          // per item (s, c): [F][n_s] moments A (24 NA), dU/dD, dq/dD (ndes each),
                             // at F (C atom0_s + c n_s)
    int F;                   // 24 NA + 2 ndes
    float *qbuf;             // [n_total][C16] corrected charges q'
    int C16;                 // candidates rounded up to 16
    float *ybuf;             // per item: [ncomp][n_s] pair-matrix products, at ncomp (C atom0_s + c n_s)
    double *iscal;           // [S][C][2]: sum U_i, sum q_i
};

// Extra arguments of the adjoint launch (gradient of the loss with respect to theta).
struct AdjArgs {
    const float *forces;     // [C][3][n_total] forces of the forward launch
    const double *rmse;      // [C][4] RMSE_e, RMSE_f, RMSE_Q of each candidate
    double lam[5];           // loss weights
    double nf;               // number of force components, 3 sum_s N_s
    float *grow;             // [S][C][n_theta] gradient of each work item
    float *scratch;          // per slot: batch_adj_floats(...) x max_atoms
};

// per-atom floats of the adjoint scratch: D, A, gU, gq (forward phases), B, B', A',
// nu (tangents), h, z' , zeta, tau (network), D-bar, nu-bar
__host__ __device__ inline int64_t batch_adj_floats(int T, int NR, int NA, int NB, int H) {
    const int ndes = NR + 4 * NA;
    return 3 * ndes + 24 * NA + 2 * T * NB + 24 * NA + ndes + 4 * H + 2 * ndes;
}

constexpr int BATCH_CLASSES = 4;        // size classes: < 48, < 128, < 384, >= 384 atoms
constexpr int BATCH_MAX_SLOTS = 1024;   // resident workgroups of the persistent launch
constexpr int BATCH_ADJ_SLOTS = 512;    // resident workgroups of the adjoint launch

inline int batch_class(int n) { return n < 48 ? 0 : (n < 128 ? 1 : (n < 384 ? 2 : 3)); }

// Host-side plan of the prepared batch (kept by the model handle).
struct BatchPlan {
    bool ready = false;
    const void *ws = nullptr;
    size_t need = 0;
    int S = 0, C_max = 0, ncomp = BATCH_COMP_FORCE, max_atoms = 0, capR = 0;
    int64_t n_total = 0, n_tiles = 0, ph_total = 0, k_total = 0, mat_total = 0, per_slot = 0;
    double qtot = 0.0;
    std::vector<BatchStruct> st;
    std::vector<int> order;
    int cls_lo[BATCH_CLASSES] = {0, 0, 0, 0}, cls_hi[BATCH_CLASSES] = {0, 0, 0, 0};  // range of `order` per class
    int groups[BATCH_CLASSES] = {8, 4, 2, 1};              // lanes per atom per class
    int slots_per_cu = 2;
    int cus = 256;
    // device pointers into the workspace
    int32_t *flags = nullptr;
    int *counter = nullptr;
    BatchStruct *st_d = nullptr;
    int *order_d = nullptr;
    int *ts = nullptr, *cntR = nullptr, *cntA = nullptr, *kcount = nullptr;
    float4 *list = nullptr, *kv = nullptr;
    float2 *ph = nullptr;
    float *mats = nullptr, *scratch = nullptr;
    double *stats = nullptr;
    float *persist = nullptr, *qbuf = nullptr, *ybuf = nullptr;
    double *iscal = nullptr;
    int F = 0, C16_max = 0;
    // gradient buffers (QNEP_BATCH_GRADIENT)
    bool grad = false;
    int64_t per_slot_adj = 0;
    float *fbuf = nullptr, *grow = nullptr, *adj_scratch = nullptr;
    double *rmse = nullptr;
    int n_slots() const {
        int s = cus * slots_per_cu;
        return s < BATCH_MAX_SLOTS ? s : BATCH_MAX_SLOTS;
    }
};

hipError_t batch_setup(const BatchStruct *st, int S, int64_t n_total, int64_t n_tiles, int64_t ph_total,
                       const float *pos, const int *type, int T, float rcR, float rcA, float4 *list, int *cntR,
                       int *cntA, int capR, int *ts, int32_t *flags, const qnep_es_params &es, float4 *kv,
                       int *kcount, float2 *ph, int ncomp, float *mats, hipStream_t stream);
bool batch_supported(int T, int NR, int NA, int NB);
hipError_t batch_eval(const BatchArgs &a, int T, int NR, int NA, int NB, int n_slots, int item_begin,
                      int item_end, int4 groups, hipStream_t stream);
hipError_t batch_loss(const double *stats, const double *E_ref, const float *thetas, int64_t n_theta, int S, int C,
                      double qtot, const double *lam, double *loss, double *rmse, hipStream_t stream);
hipError_t batch_adjoint(const BatchArgs &a, const AdjArgs &g, int T, int NR, int NA, int NB, int n_slots,
                         int4 groups, hipStream_t stream);
hipError_t batch_grad_reduce(const float *grow, const float *thetas, int64_t n_theta, int S, int C, double l1,
                             double l2, float *dthetas, hipStream_t stream);

}  // namespace qnep
