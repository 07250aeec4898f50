// Host-side structures of the ChFSI library shared by the driver translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <functional>
#include <vector>

#include "chfsi.h"
#include "common.h"

// Grow-only device arena.  A first pass with `measuring` set sums the sizes of a buffer layout;
// the second pass carves the buffers out of one allocation.
struct Arena {
    char* base = nullptr;
    size_t cap = 0, off = 0;
    bool measuring = false, failed = false;
    void grow(size_t bytes);
    void* get(size_t bytes);
    template <class T> T* take(size_t count) { return (T*)get(count * sizeof(T)); }
    void begin(bool measure) { off = 0; measuring = measure; failed = false; }
};

// Grow-only pinned host buffer (hipHostMalloc), released by chfsi_destroy.
struct PinBuf {
    char* p = nullptr;
    size_t cap = 0;
    bool reserve(size_t bytes);
    void release();
};

enum { PH_REDUCE = 0, PH_LANCZOS, PH_FILTER, PH_QR, PH_RR, PH_RESID, PH_LOCK, PH_BACK, PH_TOTAL, NPHASE };

// hipEvent pairs per phase, summed after the final synchronisation of a solve
struct PhaseTimer {
    struct Span { int phase; hipEvent_t b, e; };
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<Span> spans;
    hipEvent_t open[NPHASE] = {};
    ~PhaseTimer();
    void mark(int phase, hipStream_t s, bool begin);
    void collect(double* out);
};

// hipEvents of every filter step: the start of its first kernel, the end of its main kernel and the
// end of its last kernel (set by the launcher from the dispatches' own timestamps, see
// GemmWs::ev_start); summed after the solve's final synchronisation
struct KernelTimer {
    struct Rec { int n, ncols, prec; int plan[4]; };
    std::vector<hipEvent_t> pool;
    std::vector<Rec> recs;                    // one per begin/end pair
    std::vector<double> log;                  // rows of the last collect (see chfsi_filter_launch_log)
    size_t used = 0;
    bool enabled = true;
    ~KernelTimer();
    // hands the step's three events and the slot of its plan to the launcher through gs (all null
    // when timing is off); end() after the launch
    void begin(int n, int ncols, int prec, GemmWs& gs);
    void end(const GemmWs& gs);
    double collect(int* launches, double* step_ms = nullptr);   // main-kernel ms; resets
};

struct TuneEntry { int prec, n, m; int bm, bn, ksplit, mode; };

// A stream of the batched solver: each problem is bound to one lane so that the small dense steps
// of different problems can overlap on the device.
struct Lane {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    // handle through which one host thread runs the dense steps of the lane's problems: the lane's
    // stream, its own split-K counters, read-only copies of the tuned plans and the degree model
    chfsi_handle sub = nullptr;
};

// A captured filter graph of the batched solver: `steps` persistent launches reading their work
// lists from a device table (see batched.hip).
struct BatchGraph {
    int steps = 0, bm = 0, bn = 0, grid = 0;
    void* table = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct chfsi_handle_s {
    int device = 0;
    hipStream_t stream = nullptr;
    Arena ws;
    Arena lob;                     // LOBPCG blocks beyond the solver workspace
    // Cholesky factor of the last overlap chfsi_solve factored: a copy of that S (n^2), its L (n^2)
    // and the inverses of L's diagonal blocks; reused when the next S is equal element for element
    Arena fc;
    int fc_n = 0;                  // order of the cached factor (0: none)
    bool fc_enabled = true;        // off for the lane handles of the batched solver
    PhaseTimer timer;
    std::vector<double> trace;
    float* model = nullptr;        // device: MLP parameters followed by 10 normalisation constants
    int* tile_cnt = nullptr;       // device: split-K arrival counters, zero between launches
    int tile_cnt_len = 0;
    KernelTimer ktimer;            // per-launch events around filter steps
    std::vector<TuneEntry> plans;  // autotuned filter-step plans
    double last_kernel_ms = 0;     // filter-step launch time of the last solve / filter call
    int last_kernel_launches = 0;
    bool has_model = false;
    PinBuf pin;                    // pinned staging of single solves
    // batched solves
    std::vector<Lane> lanes;
    std::vector<Arena> barena;     // one device arena per problem
    std::vector<PinBuf> bpin;      // one pinned staging buffer per problem
    std::vector<BatchGraph> graphs;
    hipStream_t cap_stream = nullptr;   // graphs are captured here (never the null stream)
    void* btable = nullptr;        // device: step tables of the batched filter
    size_t btable_cap = 0;
    PinBuf btable_host;
    int batch_bm = 64, batch_bn = 64;   // tile of the persistent filter kernel
    // per-problem tiles: (n, m, bm, bn) entries; when batch_mixed, every problem of a step takes the
    // tile of its (n, m) (else batch_bm x batch_bn) in the kernel with a tile per problem
    bool batch_mixed = false;
    std::vector<std::array<int, 4>> batch_tiles;
    double batch_filter_ms = 0, batch_flops = 0;
    int batch_graph_launches = 0, batch_kernel_launches = 0;
    bool batch_use_graph = true;   // replay each loop's filter steps as one captured graph
    int batch_lanes = 3;           // streams (and host threads) the dense steps of a batch are spread over
    hipEvent_t bev[3] = {nullptr, nullptr, nullptr};   // filter start / end, lane join
};

// steps (solver.hip)
chfsi_status step_reduce(chfsi_handle h, int n, const zd* A, int lda, const zd* S, int lds, zd* H, zd* L, zd* dinv,
                         zd* hwork, int* info_dev, const GemmWs& gw);
// L L^H = S (L lower, zero above the diagonal, dinv the inverses of its 64 x 64 diagonal blocks);
// the factorisation's info is copied to info_host (valid after a synchronisation)
chfsi_status step_factor_enqueue(chfsi_handle h, int n, const zd* S, int lds, zd* L, zd* dinv, int* info_dev,
                                 int* info_host, const GemmWs& gw);
chfsi_status step_reduce_enqueue(chfsi_handle h, int n, const zd* A, int lda, const zd* S, int lds, zd* H, zd* L,
                                 zd* dinv, zd* hwork, int* info_dev, int* info_host, const GemmWs& gw);
chfsi_status step_lanczos_enqueue(chfsi_handle h, int n, const zd* H, int ldh, int k, unsigned long long seed,
                                  zd* LV, zd* w, zd* c, double* coef_dev, double* hal, double* hbe);
chfsi_status lanczos_finish(int k, const double* hal, const double* hbe, std::vector<double>& theta,
                            std::vector<double>& z1sq, double& beta_k, int& k_used);
chfsi_status step_lanczos(chfsi_handle h, int n, const zd* H, int ldh, int k, unsigned long long seed, zd* LV, zd* w,
                          zd* c, double* coef_dev, std::vector<double>& theta, std::vector<double>& z1sq,
                          double& beta_k, int& k_used);
chfsi_status step_orthonormalize(chfsi_handle h, int n, int ma, zd* Y, int ldy, int nl, const zd* YL, int ldyl,
                                 zd* G, zd* Cm, zd* dinv, double* dsc, int* info_dev, const GemmWs& gw,
                                 double* host_tmp = nullptr, zd* T = nullptr);
chfsi_status step_rayleigh_ritz(chfsi_handle h, int n, const zd* H, int ldh, int ma, zd* Y, int ldy, zd* HY, zd* T,
                                zd* G, double* theta_dev, double* r_dev, void* eig_work, double* eig_host,
                                const GemmWs& gw, PhaseTimer* tm, double eig_stop = 0.0);
void filter_coefficients(int dmax, double a, double b, double mu1, std::vector<FilterStep>& steps);
FilterStep filter_step_coefficients(int k, double a, double b, double mu1, double& sigma);
// The filters: hy0 (nullable, complex128, ld n) = H times the block's columns in their order, which
// makes step 1 an elementwise update instead of a product.
chfsi_status filter_f64(chfsi_handle h, int n, const zd* H, int ldh, int ma, zd* Y, int ldy, zd* T,
                        const std::vector<int>& deg, double a, double b, double mu1, int* flag_dev, const GemmWs& gw, double& flops, long long& matvecs,
                        const zd* hy0 = nullptr);
chfsi_status filter_f32(chfsi_handle h, int n, const zf* Hf, int ldh, int ma, zf* Yf, int ldy, zf* Tf,
                        const std::vector<int>& deg, double a, double b, double mu1, int* flag_dev, const GemmWs& gw, double& flops, long long& matvecs,
                        const zd* hy0 = nullptr);
void host_tridiag_eig(int k, const double* al, const double* be, std::vector<double>& theta,
                      std::vector<double>& z1sq);

chfsi_status filter_bf16(chfsi_handle h, int n, const uint16_t* Hb, int ldh, int nterms, int ma, zf* Yf, int ldy,
                         zf* Tf, uint16_t* ysplit, const std::vector<int>& deg, double a, double b, double mu1,
                         int* flag_dev, const GemmWs& gw, double& flops, long long& matvecs, const zd* hy0 = nullptr);
// degree network (mlp.hip)
chfsi_status learned_degrees(chfsi_handle h, int ma, const double* theta_dev, const double* r_dev, double a,
                             double b, double mu1, double thr, const std::vector<int>& dprev, float* feat,
                             float* dpred, int* iscr, int dmin, int dmax, int* out,
                             const std::function<int(int)>& fallback);

// tuned plan for a filter step (tune.hip); leaves gw unchanged when the table has no entry
void apply_tuned_plan(chfsi_handle h, int prec, int n, int ncols, GemmWs& gw);

// extra small kernels (blas1.hip)
int launch_zero_upper(hipStream_t s, int n, zd* L, int ldl);
int launch_add_diag_const(hipStream_t s, int m, zd* G, int ldg, double shift);
