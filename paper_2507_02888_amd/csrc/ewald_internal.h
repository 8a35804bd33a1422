// Internal layout shared by the host set-up (ewald_host.cpp) and the HIP
// kernels (ewald_device.hip, ewald_run_d*.hip).  Not part of the public ABI.
#pragma once

#include <cstddef>
#include <cstdint>

#if defined(__HIPCC__) || defined(__HIP__)
#define EW_HD __host__ __device__
#else
#define EW_HD
#endif

namespace ewald {

constexpr int SEG = 4;            // G slots per segment: consecutive n along the last reduced index
constexpr int BLOCK = 256;        // threads per workgroup of every kernel
constexpr int MAX_CAND = 16;      // +-pairs of minimum-image candidate offsets
constexpr int MAX_COSET = 1;      // nonzero cosets of an orthogonal sublattice (index <= 2)
constexpr int HDR_BYTES = 256;    // per-walker state header
// Byte offset, in the state buffer (inside the first walker's header), of the
// fused kernel's work counter when its workgroups take walkers from a queue.
constexpr int QUEUE_OFF = 192;
constexpr int MAX_SPT = 8;        // segments per thread held in registers (MAX_SEGMENTS / BLOCK)
constexpr int TILE_P = 8;         // particles per phase-table tile when rebuilding rho (tiles are even)
static_assert(TILE_P % 2 == 0, "rebuild tiles hold whole particle pairs");
constexpr int RUN_CHUNK = 64;     // proposals staged in LDS per chunk by the fused kernel
constexpr int WTAB_MAX = 1024;    // largest shell table kept in LDS by the fused kernel
constexpr int POLY_MAX = 32;      // largest degree of the pair-potential polynomial (FP64)
constexpr int POLY32_MAX = 22;    // largest degree of its FP32 counterpart
constexpr int UDEG = 15;          // degree of the Jastrow u polynomial in t = r / L_u (N_u + C <= UDEG)

// Per-walker state header (first bytes of the walker's state block).
struct WalkerHdr {
  int32_t counter;      // accepted moves since rho was last rebuilt
  int32_t pending_k;    // -1: no pending move
  int32_t n_accepts;
  int32_t n_refresh;
  double pending_s[3];  // wrapped fractional position of the pending move
  double drift_max;     // max |rho_running - rho_rebuilt| (bits updated with atomicMax)
};
static_assert(sizeof(WalkerHdr) <= QUEUE_OFF && QUEUE_OFF + 4 <= HDR_BYTES, "header too large");

// One system as the kernels see it (lives in device memory).
struct DevSys {
  int dim;
  int n_mobile;
  int n_fixed;
  int n_seg;            // segments of SEG slots
  int nmax[3];          // largest |n_d| over the G set
  int nm;               // max(nmax): phase tables hold n in [-nm, nm]
  int n_cand;           // +-pairs of candidate offsets
  int has_jastrow;
  int refresh_every;
  int precision;        // 0 FP64, 1 FP32-mixed
  int poly_deg;         // 16 or 32: degree of p64 (p32 uses 12 or 22)
  double A[9];          // lattice rows a_i (row-major 3x3)
  double Ainv[9];       // s = r Ainv for row vectors
  double Lrot[9];       // the lattice rotated to lower-triangular form (distances only)
  double alpha;
  double rc2;           // r_cut^2
  double poly_scale;    // 2 / r_cut^2: t = r^2 poly_scale - 1 maps [0, r_cut^2] to [-1, 1]
  double e_const;       // E_self + E_background + fixed-ion real-space energy
  double cand[MAX_CAND][4];  // (v_x, v_y, v_z, |v|^2) of one of each +-pair, rotated frame
  // Orthogonal-sublattice frame (ortho = 1): the lattice contains mutually
  // orthogonal vectors of lengths box[d] spanning a sublattice of index
  // n_coset + 1 <= 2 whose nonzero coset is offset by half box sides.
  // Positions in this frame are x = s F; the minimum image is a per-axis wrap
  // into the box and min(|x|^2, |x|^2 + cc - sum_d cw[d] |x_d|) (cc = +inf
  // when there is no coset).
  int ortho;
  int n_coset;
  double F[9];
  double box[3];
  double ibox[3];
  double cw[MAX_COSET][3];  // box[d] where the coset has a half-box offset along d, else 0
  double cc[MAX_COSET];     // sum over those d of box[d]^2 / 4 (+inf: no coset)
  // Jastrow derivatives: reciprocal lattice rows b_d (G = sum_d n_d b_d) and
  // jlap_c = sum_{G in H} a_s(G) |G|^2
  double B[9];
  double jlap_c;
  // Jastrow two-body polynomial term u (has_u): u(r) = sum_m c_m t^m for
  // t = r / L_u < 1, with c = u_c0 for a pair of equal spin labels and
  // u_c0 + u_dc for unequal ones (the set-up expands the product form of the
  // term into powers of t); mobile particles only.
  int has_u;
  double u_cut2;          // L_u^2
  double u_icut;          // 1 / L_u
  double u_c0[UDEG + 1];
  double u_dc[UDEG + 1];
  const int32_t* spin;    // [n_mobile] spin labels (0/1)
  // frame axes as rows (Cartesian unit vectors): Eo of the orthogonal
  // sublattice frame (x = s F), El of the lower-triangular frame (Lrot), so
  // that a displacement x in a frame is sum_d x_d E[d] in Cartesian axes
  double Eo[9];
  double El[9];
  // Layered 2D system (n_layers = 2): mobile particles j >= n0 and the ions
  // with fixed_layer 1 lie in the second plane, dz2 = (z_1 - z_0)^2 apart;
  // rho of the second plane follows the first in the walker state
  // (SEG n_seg slots later); wx: the cross-plane weight per slot,
  // rho_fix1: the second plane's ions.
  int n_layers;
  int n0;
  double dz2;
  const double* wx;
  const double* wx_tab;   // [n_wtab] the cross-plane weight per shell (0 for padding)
  const double* rho_fix1;
  const int32_t* fixed_layer;
  // erf(alpha r)/(alpha r) = sum_i p64[i] t^i for r < r_cut (p32: FP32 copy of lower accuracy)
  double p64[POLY_MAX + 1];
  float p32[POLY32_MAX + 1];
  // device tables (slot-planar: slot j of segment s lives at j * n_seg + s)
  const uint32_t* seg_n;     // [n_seg] packed n of the segment's first slot (int8 x3)
  const double* w;           // [SEG * n_seg] weight, 0 for padding
  const double* ja;          // [SEG * n_seg] Jastrow coefficient, or nullptr
  const double* rho_fix;     // [SEG * n_seg][2] fixed-ion structure factor
  const uint16_t* slot_shell;  // [SEG * n_seg] index into wa_tab (n_wtab - 1 for padding)
  const double* wa_tab;      // [n_wtab][2] (weight, Jastrow coefficient) per shell
  const double* jg2_tab;     // [n_wtab] Jastrow coefficient times |G|^2 per shell (0 for padding)
  int n_wtab;                // n_shells + 1 (a zero entry for padding slots)
  int wtab_lds;              // 1 if n_wtab <= WTAB_MAX: the fused kernel reads wa_tab from LDS
  const double* fixed_s;     // [n_fixed][dim] wrapped fractional ion positions
  const double* fixed_q;     // [n_fixed]
  const double* mobile_q;    // [n_mobile]
};

// Walker descriptors are uploaded in launch order: most expensive first (a
// longest-processing-time order), so that with one workgroup per walker the
// hardware dispatcher starts the large walkers of an uneven batch early and
// the tail is made of small ones.  `id` is the walker's index in the caller's
// arrays.
struct DevWalker {
  int sys;
  int n_mobile;
  long long state_off;  // byte offset of the walker's state block
  long long pos_off;    // first row in the packed position input
  int id;
  int pad_;
};

EW_HD inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

EW_HD inline size_t walker_pos_bytes(int n_mobile, int dim) { return align256(size_t(n_mobile) * dim * 8); }
// rho of a layered system holds one block of n_seg SEG slots per plane
EW_HD inline size_t walker_rho_bytes(int n_seg, int n_layers) {
  return align256(size_t(n_seg) * SEG * 16 * size_t(n_layers > 1 ? n_layers : 1));
}
EW_HD inline size_t walker_state_bytes(int n_mobile, int dim, int n_seg, int n_layers = 1) {
  return HDR_BYTES + walker_pos_bytes(n_mobile, dim) + walker_rho_bytes(n_seg, n_layers);
}

inline uint32_t pack_n(int a, int b, int c) {
  return uint32_t(a & 0xff) | (uint32_t(b & 0xff) << 8) | (uint32_t(c & 0xff) << 16);
}

// ---- launch interface implemented in ewald_device.hip -----------------------

struct LaunchBatch {
  const DevSys* d_sys;      // device array [n_sys]
  const DevWalker* d_walk;  // device array [n_walkers]
  int n_walkers;
  int dim;
  int mixed;
  int has_jastrow;          // any system with Jastrow coefficients or a u term
  int has_u;                // any system with a Jastrow u term
  int layered;              // any layered 2D system (the fused kernels with a second plane serve the sweep)
  int max_n_seg;
  int max_nm;
  int max_particles;        // max n_mobile over systems
  int max_fixed;
  int refresh_every;        // max over systems (0: no rebuild kernel needed)
  int poly_deg;             // max pair-polynomial degree over systems (16 or 32)
  int max_wtab;             // largest LDS shell table over systems (0: none in LDS)
  int all_wtab_lds;         // every system's shell table fits in LDS
  int all_ortho;            // every system has an orthogonal-sublattice frame (DevSys::ortho)
  int run_threads;          // fused kernel: workgroup size (0: default for the segment count)
  int run_waves;            // fused kernel, 256 threads: waves per SIMD it is compiled for (0: 2)
  int run_chunk;            // fused kernel: moves per chunk (0: as many as LDS allows, <= RUN_CHUNK)
  int run_wpb;              // fused kernel: walkers per workgroup taken from a queue (0: one
                            // walker per workgroup, dispatched by the hardware)
  int n_cu;                 // compute units of the device
  int general_frame;        // fused kernel: 1 = general minimum-image reduction even if all_ortho
};

// The fused kernel's launch shape for a batch (all zero: it does not fit and
// the per-step kernels run instead).
struct RunPlan {
  int fused;          // 1 if the fused kernel runs
  int threads;        // workgroup size
  int spt;            // segments per thread
  int ppr;            // particles per thread held in registers
  int chunk;          // moves per chunk
  int general_frame;  // 1 = general minimum-image reduction
  int lds_bytes;
  int blocks_per_cu;  // workgroups per CU allowed by registers
  int waves;          // 256 threads: waves per SIMD the kernel is compiled for (512 / waves registers
                      // per lane); 0 for the other shapes (their bound is fixed)
  int walkers_per_block;  // 0: one walker per workgroup; else the queue mode's walkers per workgroup
  int grid;               // workgroups launched
};

// Each returns 0 on success or the hipError_t of the failed launch.
int launch_energy(const LaunchBatch& b, const double* pos, char* state, double* energy,
                  double* jastrow, void* stream);
// jgrad/jlap (both or neither): gradient [W][dim] ([S][W][dim] for launch_run)
// and Laplacian of the Jastrow value with respect to the moved particle at the
// proposed configuration.
int launch_delta(const LaunchBatch& b, char* state, const int32_t* k, const double* new_pos,
                 double* delta, double* djastrow, double* jgrad, double* jlap, void* stream);
int launch_accept(const LaunchBatch& b, char* state, const uint8_t* accept, void* stream);
// accept_prev != NULL: the accept of the pending move folded into the delta
// of the next (NULL: launch_delta).
int launch_step(const LaunchBatch& b, char* state, const uint8_t* accept_prev, const int32_t* k,
                const double* new_pos, double* delta, double* djastrow, double* jgrad, double* jlap,
                void* stream);
int launch_run(const LaunchBatch& b, char* state, int n_steps, const int32_t* k,
               const double* new_pos, const uint8_t* accept, double* delta, double* djastrow,
               double* jgrad, double* jlap, void* stream);

void plan_run(const LaunchBatch& b, RunPlan* plan);
bool run_threads_valid(int max_n_seg, int threads);
// Warm-up plus `reps` timed fused launches on `stream` (synchronises); best time in ms.
int time_run(const LaunchBatch& b, char* state, int n_steps, const int32_t* k, const double* new_pos,
             const uint8_t* accept, double* delta, void* stream, int reps, float* best_ms);

// Device memory helpers (ewald_device.hip); return 0 on success.
int dev_alloc(void** p, size_t bytes);
int dev_free(void* p);
int dev_upload(void* dst, const void* src, size_t bytes);
int dev_current(int* device);
int dev_cu_count(int* n_cu);  // compute units of the current device
const char* dev_error_string(int code);
int dev_arch(char* buf, int len);  // the current device's architecture name
int dev_memset(void* p, int value, size_t bytes);
int dev_copy(void* dst, const void* src, size_t bytes);  // device to device, synchronous
int stream_sync(void* stream);  // waits for the work queued on `stream`

// Event pairs for the per-call timers (ewald_device.hip); return 0 on success.
int event_pair_create(void** pair);
int event_pair_record(void* pair, int which, void* stream);  // which: 0 start, 1 end
int event_pair_elapsed(void* pair, float* ms);                // waits for the end event
void event_pair_destroy(void* pair);
int stream_capturing(void* stream, int* capturing);

// Per-call timer (enabled by EWALD_TIMING=1 or ewald_timing_enable): counts
// the call, its host time and, outside graph capture, the GPU time between
// two events recorded on its stream around it.  One per ABI call that
// launches work, constructed first thing in the call.
class CallTimer {
 public:
  CallTimer(const char* name, void* stream) noexcept;
  ~CallTimer();
  CallTimer(const CallTimer&) = delete;
  CallTimer& operator=(const CallTimer&) = delete;

 private:
  const char* name_;
  void* stream_;
  void* pair_ = nullptr;
  bool on_ = false;
  double t0_ = 0.0;
};

}  // namespace ewald
