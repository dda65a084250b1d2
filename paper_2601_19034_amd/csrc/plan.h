// Per-call plan: sizes derived on the host and device pointers into the workspace.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/qnep.h"
#include "common.h"

namespace qnep {

// pipeline stages timed by qnep_model_enable_timing (names in api.cpp)
enum Stage : int {
    ST_SORT = 0, ST_LISTS, ST_LISTS_C, ST_DESC, ST_MLP, ST_REAL, ST_EWALD_SK, ST_EWALD_ATOMS, ST_SPREAD,
    ST_FFT_FWD, ST_INFLUENCE, ST_FFT_INV, ST_GATHER, ST_PHI, ST_RADIAL, ST_ANG, ST_ASSEMBLE,
    ST_FINAL, ST_OTHER
};

struct Timer;

// reverse-mode state (qnep_backward)
struct Backward {
    double gE = 0.0, gP[3] = {0.0, 0.0, 0.0};
    float *dpos = nullptr, *dtheta = nullptr;  // caller outputs (may be null)
    double *dcell = nullptr;
    float *Fout = nullptr, *Zout = nullptr;    // forward outputs kept in the workspace
    double *energy = nullptr, *virial = nullptr, *pol = nullptr, *terms = nullptr;
    float *Xvec = nullptr, *delta = nullptr, *Gam = nullptr, *Gc = nullptr;
    double *sums = nullptr, *sW0 = nullptr, *sVec = nullptr, *sCR = nullptr, *sCA = nullptr;
    double *partials = nullptr;
};

struct Plan {
    // ---- model
    int N = 0, T = 0, NR = 0, NA = 0, NBR = 0, NBA = 0, LMAX = 4, H = 0, ndes = 0;
    double rcR = 0, rcA = 0;
    int mlp_prec = QNEP_MLP_FP32;
    int64_t off_cR = 0, off_cA = 0, off_nn = 0, per_species = 0, off_b1E = 0, off_s = 0, n_theta = 0;
    // ---- electrostatics
    int mode = 1, method = 0, kinc = 0, order = 5;
    int iso = 0;  // isolated system: no periodic images, direct Coulomb sum, Born charges of Eq. 27
    double alpha = 0.3, rc_coul = 9.0, kmax = 0, qtot = 0;
    float efield[3] = {0.f, 0.f, 0.f};  // external field (V/Angstrom)
    int mesh[3] = {0, 0, 0};
    int64_t mesh_pts = 0;
    Cell cell;
    double vol = 0;
    // ---- binning and lists
    int nc[3] = {1, 1, 1};
    int ncell = 1;
    int mR[3] = {1, 1, 1}, mC[3] = {1, 1, 1};
    int capR = 0, capA = 0;
    int nblk = 0;  // blocks of RED_THREADS threads over N
    // ---- Ewald
    int nk_box[3] = {0, 0, 0};
    int64_t nk_cap = 0;      // capacity of the half k-set
    int row_cap = 0;         // rows (n0, n1) of the k box: an upper bound of the nonempty rows
    int NZP = 0;             // n2 entries per row in the structure-factor and phase tables (16 | NZP)
    int NZ4 = 0;             // n2 entries per row in the per-atom product (even)
    int s_chunks = 0, s_chunk = 0;  // atom chunks (count, atoms) of the structure-factor product
    int r_chunks = 0, r_chunk = 0;  // row chunks (count, rows) of the per-atom product
    // ---- device workspace
    int32_t *flags = nullptr;
    double *scalars = nullptr;
    double *partials = nullptr;
    int64_t partials_cap = 0;
    double *red_tmp = nullptr;  // per-slice sums of one partials reduction
    int *cid = nullptr, *cell_count = nullptr, *cell_start = nullptr, *cell_cursor = nullptr, *perm = nullptr;
    int *scan_tmp = nullptr;
    float4 *xyzt = nullptr;  // sorted positions (x, y, z) with the species in w (as int bits)
    float4 *xyzq = nullptr;  // sorted positions with the corrected charge q' in w (real-space sum)
    int *ts = nullptr;       // sorted species
    uint32_t *listR = nullptr, *listA = nullptr;
    int *cntR = nullptr, *cntA = nullptr;
    float *D = nullptr, *Amom = nullptr;
    float *Bsum = nullptr;  // per-species radial basis sums (backward only)
    float *U = nullptr, *qraw = nullptr, *gU = nullptr, *gq = nullptr;
    float *phi = nullptr, *Fst = nullptr, *hT = nullptr;
    float *pairFA = nullptr;  // angular pair buffer [i][capA][2] float4: F_ij, then a_ij
    float *Fnep = nullptr, *Znep = nullptr;
    float *Vat = nullptr;  // per-atom virial, symmetric parts [6][N] (xx yy zz xy xz yz), sorted order
    float *Siso = nullptr; // isolated systems: sum_j (a_ji - a_ij) per atom [3][N], sorted order
    float4 *kvec = nullptr;   // (kx, ky, kz, G) of the half set
    int *kcount = nullptr;
    int4 *krows = nullptr;    // nonempty rows of the half set: (n0, n1, first n2, count)
    int *krowoff = nullptr;   // index of each row's first wave vector
    int *knrows = nullptr;    // number of nonempty rows
    float2 *ewX = nullptr, *ewY = nullptr, *ewZ = nullptr;  // phase tables [entry][N]
    float *Spart = nullptr;   // [s_chunks][row_cap][NZP][re, im]
    float2 *Ubox = nullptr;   // [row_cap][4][NZ4]: G S, k_x G S, k_y G S, k_z G S
    float *ephi = nullptr;    // [r_chunks][4][N]: partial potential and force sums
    float2 *Sk = nullptr;     // [nk_cap]
    bool bricks = false;      // charge assignment by mesh bricks (else global atomics into rho)
    int brickP[3] = {0, 0, 0}, brickNb[3] = {0, 0, 0};
    float *rho = nullptr;
    float2 *meshA = nullptr;   // rho, then its transform S
    float2 *meshAB = nullptr;  // the two packed spectra / fields, interleaved [point][2]
    float2 *meshV = nullptr;   // per-atom virial: three packed spectra / fields [3][point]
    // ---- call arguments
    const float *pos = nullptr;
    const int32_t *type = nullptr;
    const float *theta = nullptr;
    qnep_outputs out{};
    hipStream_t stream = nullptr;
    Timer *timer = nullptr;
    Backward bw;
};

// records the end of `stage` (work enqueued since the previous mark) when timing is on
void stage_mark(const Plan &p, int stage, int launches = 1);

// module launchers (each returns hipSuccess or the first launch error)
hipError_t launch_neighbors(const Plan &p);
hipError_t launch_descriptors(const Plan &p);
hipError_t launch_mlp(const Plan &p);
hipError_t launch_charges(const Plan &p);
hipError_t launch_real_space(const Plan &p);
hipError_t launch_direct_coulomb(const Plan &p);
hipError_t launch_centroid(const Plan &p);
hipError_t launch_ewald(const Plan &p);
size_t ewald_atoms_lds_bytes(int NZ4);  // dynamic LDS of the per-atom Ewald product
hipError_t launch_pppm(const Plan &p);
// mesh bricks of the charge assignment: edge P (points) and count nb per axis
struct BrickGeom {
    int P[3], nb[3];
};
bool spread_bricks(const int *mesh, const int *nc, BrickGeom *bg);
hipError_t launch_forces(const Plan &p);
hipError_t launch_finalize(const Plan &p);
hipError_t launch_zero_outputs(const Plan &p);

hipError_t launch_backward(const Plan &p);

// fixed-order reduction of partials[nblk][nv] into scalars[slot..slot+nv)
hipError_t reduce_partials(const Plan &p, int nblk, int nv, int slot, bool accumulate);
// the same into an arbitrary FP64 destination
hipError_t reduce_partials_to(const Plan &p, int nblk, int nv, double *dst);
// fills n floats/ints with zero (a kernel, not a memset, so that the sequence can be captured)
hipError_t fill_zero(void *ptr, size_t bytes, hipStream_t s);

// in-house 3D FFT (complex, in place on `data` using `tmp` as scratch); sign -1 forward, +1 inverse
hipError_t fft3d(float2 *data, float2 *tmp, const int *mesh, int sign, hipStream_t s, int inner = 1);
bool fft_length_supported(int n);

}  // namespace qnep
