// Device-resident solver state and kernel argument blocks of the single-signal path.
#pragma once
#include <stdint.h>

namespace ds {

enum TestKind { TEST_NONE = 0, TEST_SAFE = 1, TEST_DST3 = 2, TEST_DOME = 3 };
enum RuleKind { RULE_ISTA = 0, RULE_FISTA = 1, RULE_SPARSA = 2, RULE_CP = 3 };
constexpr int BB_MEM_MAX = 15;  // SpaRSA: earlier iterates kept in the acceptance memory

// Every scalar of the iteration lives in device memory so that a whole chunk of
// iterations can be enqueued (or graph-replayed) without host round trips.
struct alignas(16) SolverState {
  // problem scalars (set up on the device)
  double lam;          // absolute penalty
  double lam_ratio;    // lambda / lambda_* when the penalty is relative, else <= 0
  double lam_max;      // lambda_*
  double L;            // step constant (backtracking: the current L_t)
  double bt_eta;       // backtracking: growth factor of L on a rejected step (0: constant step)
  double yy;           // ||y||^2
  double rho2;         // ||y/lambda - c||^2 of the sphere centre (0 for SAFE)
  double alpha;        // DST3/DGST3: c = y/lambda - alpha * n
  double nn;           // ||n||^2 (n = d_* or D_g* D_g*^T y / lambda_*)
  double ny;           // n^T y
  double marg_slack;   // bound on the FP64 rounding error of the margins
  double gamma_z;      // relative rounding bound of one streamed dot product
  double kappa_z;      // max_i ||d_i|| (Lasso) or max_g ||D_g||_F / w_g: scales the slack
  double gap_tol_abs;  // gap_tol * ||y||^2 (0: fixed iteration count)
  // per-iteration scalars
  double tt;           // ||theta||^2 (FP64 from the stored theta)
  double ty;           // theta^T y
  double zsup;         // upper bound of ||D_A^T theta||_inf (or max_g ||D_g^T theta|| / w_g)
  double omega;        // Omega(p) of the point theta was evaluated at
  double mu, gap, primal, dual;
  double r_last;       // radius of the last iteration (no slack)
  double r_min;        // smallest radius (no slack), for reporting
  double r_scr;        // screening radius in use, slack included
  double r_slack;      // slack part of r_scr
  double l_prev;       // FISTA l_{t-1}
  int32_t n_active;    // active units (atoms or groups) in the current list
  int32_t n_support;   // entries of the support list of the next primal point
  int32_t iter;        // iterations completed
  int32_t done;        // 1 once the stopping rule fired (later kernels become no-ops)
  int32_t cur;         // which active-list buffer is current
  int32_t i_star;      // arg-max atom / group of lambda_*
  int32_t nnz;         // non-zeros of x after the last update
  int32_t status;      // 0 ok, 1 trivial (lambda >= lambda_*), -1 invalid input
  int32_t max_iter;
  int32_t n_active_atoms;
  int32_t n_kept;      // units kept by the last iteration (list entries may be stale)
  int32_t compact;     // 1: the next correlation pass rewrites the list without stale entries
  int32_t pending;     // 1: a correlation pass ran whose scalars are not computed yet
  int32_t n_omp;       // Omega(p) partials the last residual pass published
  int32_t rejected;    // backtracking: the last step was rejected (x, u were restored)
  int32_t n_reject;    // backtracking: rejected steps so far
  // SpaRSA: objective at the current primal point (newest entry) and at up to bb_mem
  // earlier iterates, oldest first
  int32_t bb_mem;      // earlier iterates kept
  int32_t phi_n;       // entries in phi_mem
  int32_t bb_new;      // 1: the primal point of the next scalar stage is a new iterate
  int32_t warm;        // 1: the first pass starts from a caller's x_0 (its support is seeded)
  int32_t stop_obj;    // 1: the solve ended on the relative objective change (obj_tol)
  int32_t pad_;
  double bb_sigma;     // sufficient-decrease constant
  double phi_mem[BB_MEM_MAX + 1];
  // Chambolle-Pock: current primal and dual steps, acceleration
  double cp_tau, cp_sigma, cp_gamma;
  double obj_tol;      // > 0: also stop when |P_{t-1} - P_t| <= obj_tol P_t (the experiments' rule)
};

template <typename T, typename V, typename A>
struct SingleArgs {
  const T* D;            // N x K column-major, leading dimension ldd
  int64_t ldd;
  int32_t N, K;
  int32_t G;             // 0: Lasso; >0 groups
  int32_t test, rule;
  int32_t par;           // iteration parity (host-known): selects the state / partial buffers
  int32_t grid_corr;     // blocks of the correlation launch whose outputs this kernel reads
                         // (= its support segments); the host shrinks the correlation grid
                         // between chunks as the active list shrinks
  int32_t nsg_prev;      // residual pass: Omega partials the previous residual pass published
  const int64_t* gptr;   // device copy of group offsets (G+1), NULL for the Lasso
  const double* w;       // device group weights (G)
  const V* y;            // observation (16-byte aligned copy)
  SolverState* st;       // two states, indexed by parity
  int32_t* act[2];       // active unit lists (double buffered)
  double* act_m[2];      // margins of the list entries (same layout as act)
  V* x;                  // primal x, dense K (atom indexed)
  V* u;                  // FISTA auxiliary u, dense K (ISTA: u == x)
  V* theta;              // residual theta = D p - y
  A* partial;            // residual partial sums, [item][npad]
  int64_t npad;
  double* z0;            // D^T y (FP64), K
  double* g;             // D^T n (FP64), K
  double* nu;            // atom norms ||d_i||, K
  double* fro;           // group Frobenius norms (G), or NULL
  double* gnorm;         // group spectral norms ||D_g||_2 (G), or NULL
  double* marg;          // margins (K for the Lasso, G for groups)
  double* nvec;          // d_* (Lasso) or n (groups), N, FP64
  // correlation -> residual hand-off (one segment per correlation block)
  int32_t* seg_cnt;      // kept units of the block
  int32_t* seg_atom;     // SEGCAP slots per block: atom index
  V* seg_val;            // SEGCAP slots per block: new value of u
  double* urec_marg;     // UCAP unit records per block: margin
  double* urec_om;       // UCAP unit records per block: |u_i| or w_g ||u_g||
  int32_t* urec_m;       // UCAP unit records per block: atoms in the unit
  double* bp0;           // correlation partials: zsup per block
  int32_t* bpi;          // 4 x MAXB: nnz, kept units, support, kept atoms per block
  // residual -> (correlation, next residual) partials, [parity]
  double* rtn;           // 2 x (2 x MAXRT): per row tile ||theta||^2, theta^T y
  double* omp;           // 2 x MAXITEM: Omega(p) per segment group
  unsigned* rt_cnt;      // per row tile arrival counters
  uint64_t* lbA;         // look-back words (list compaction)
  unsigned* counters;    // arrival / virtual-block counters
  void* tele;            // per-iteration telemetry records, or NULL
  int32_t tele_cap;
  uint64_t* kclk;        // NULL, or 2 wall-clock stamps per correlation block (start, end)
  int32_t screen_static; // 1: the radius is taken from the first iteration only
  // backtracking (bt = 1): the correlation pass keeps, per support slot, the previous x
  // and u and the step d = x' - p, so that a rejected step can be undone
  int32_t bt;
  V* seg_xo;             // SEGCAP slots per block: x before the step
  V* seg_po;             // SEGCAP slots per block: p (u, or x for ISTA) before the step
  double* seg_d;         // SEGCAP slots per block: d = x' - p (exact difference of stored values)
  double* urec_omo;      // UCAP unit records per block: Omega term of p
  double* urec_dn;       // UCAP unit records per block: ||d_unit||^2
  double* bpd;           // ||d||^2 per correlation block
  double* bpe;           // SpaRSA: z^T d + lambda (Omega(x') - Omega(p)) per correlation block
  double* rtr;           // Chambolle-Pock: 2 x MAXRT, per row tile ||D u - y||^2, [parity]
  double* dtn;           // ||D d||^2 per row tile (the check pass)
};

// Per-iteration telemetry written by the last correlation block.
struct TeleRec {
  int32_t n_atoms;
  int32_t n_units;
  int32_t n_support;
  int32_t nnz;
  double r;
  double gap;
};

}  // namespace ds
