// pdmi_internal.h -- device data layout and kernel launchers of the peridynamics library.
//
// Device layout (one context, all instances concatenated):
//   node records  rec[2][nn]      48 bytes per node: x (3 x f64) then u.  FP64: u as 3 x f64;
//                                 FP32: u as 3 x f32 at byte 24, bytes 36..47 unused.  Two
//                                 copies hold consecutive displacement levels (ping-pong);
//                                 x is written once into both.
//   master u      um[2][3][nn]    FP32 build only: the f64 displacement the integrator
//                                 advances (the records carry its f32 rounding for the
//                                 bond arithmetic); ping-pong like the records
//   velocity      v[3][nn]        structure of arrays, f64
//   acceleration  a[3][nn]        structure of arrays, f64 (velocity Verlet)
//   sentinel      rec[*][nn]      one extra record far from every node; padding slots point at it,
//                                 followed by kRecPad zero records so the staged kernel's
//                                 fixed-size range loads stay in bounds
//   slots         col[ns]         int32 per slot in "slices": a slice is the W = 64/G nodes one
//                                 wavefront serves (G lanes per node); its slots are stored as
//                                 T rows of 64 entries, entry (t, w*G + g) = slot t*G + g of the
//                                 slice's node w.  col >= 0: intact bond to device node
//                                 col & kColNode, bit 30 (kColNoFail) set when the bond
//                                 touches a no-failure zone, bit 29 (kColSoft) once it has
//                                 softened under a damage law; col < 0: ~col is the word of
//                                 a broken bond, or the sentinel nn for padding.
//   stiffness     kslot[ns]       f64 per slot, same layout (only with a per-slot stiffness field)
//   node stiffness na[nn+1], nw[nn+1]  f64 per node (only with a per-node stiffness field,
//                                 bond stiffness sqrt(k_i k_j)): na = sqrt(k_i), nw = sqrt(k_j) V_j;
//                                 entry nn (the sentinel) is 0
//   slices        slice_ptr/T/inst first entry, row count and instance of every slice
//
// Staged layout (one lane per node, 64 nodes per slice).  The neighbours of a slice are
// covered by "ranges" of at most kSegMax consecutive device nodes; each range's slots
// are cut into "pieces" of at most kPieceRows rows of 64 uint16 entries.  A wavefront
// copies a piece's node records and entries into LDS, then reads neighbours from there.
//   pieces        int2 {first node of the range, len | T << 8} per piece
//   slice_piece   first piece of every slice (+ one past the last)
//   ent[ns]       uint16 per slot: bits 0..12 = byte offset of the neighbour's record in the
//                 staged copy (48 x index into the range; kEntPad for padding, the LDS
//                 sentinel record), bit 13 = softened, bit 14 = no-failure zone, bit 15 =
//                 broken; slice_ptr gives each slice's first entry.
//   smax[ns]      f64 per slot (with damage laws): the largest stretch the slot reached
//                 beyond its law's elastic limit (0 while it has not); cls[ns] uint8: the
//                 slot's law (bond class) when an instance has several
//                 The entry array ends with kPieceRows spare rows (whole 8-row blocks are
//                 loaded).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace pdmi {

constexpr int kWave = 64;
constexpr int kBlock = 256;             // 4 wavefronts per workgroup, one slice each
constexpr int kRowUnroll = 2;           // slot rows per step-kernel iteration; every slice's row
                                        // count is a multiple, and the slot arrays carry this
                                        // many spare rows at the end
constexpr int kSegMax = 80;             // node records per staged range (LDS slot kSegMax: sentinel)
constexpr int kPieceRows = 8;           // slot rows per staged piece
constexpr int kStageChunks = 4 * 64;    // 16-byte record chunks one staged range load covers
constexpr int kEntPad = kStageChunks * 16;  // entry byte offset of the LDS sentinel record
constexpr int kRecPad = kStageChunks / 3 + 2;  // zero records after the sentinel
// slot flags: a bond touching a no-failure zone never breaks (Secs. 5.1, 6, 7)
// and a bond that has softened under a damage law is marked so its state is read
constexpr int32_t kColNoFail = 0x40000000;  // sliced word: no-failure bit
constexpr int32_t kColSoft = 0x20000000;    // sliced word: softened bit
constexpr int32_t kColNode = 0x1fffffff;    // sliced word: neighbour index bits
constexpr uint32_t kEntOff = 0x1fff;        // staged entry: record byte offset bits
constexpr uint32_t kEntSoft = 0x2000;       // staged entry: softened bit
constexpr uint32_t kEntNoFail = 0x4000;     // staged entry: no-failure bit
constexpr uint32_t kEntBroken = 0x8000;     // staged entry: broken bit

// One damage law (bond class): stretch breakpoints s[0] < ... < s[nb-1] with force ratios
// r[0] = 1, ..., r[nb-1] = 0.  A monotonic pull follows c s up to s[0], then c s[0] times
// the interpolated ratio; the bond is broken from s[nb-1] on (nb = 1: the brittle law).
constexpr int kLawMaxB = 8;
constexpr int kLawMaxClasses = 8;
struct LawRec {
    double s[kLawMaxB];
    double r[kLawMaxB];
    double slope[kLawMaxB];  // (r[k+1] - r[k]) / (s[k+1] - s[k]) of segment k
    int32_t nb;
    int32_t pad_;
};
static_assert(3 * kSegMax <= kStageChunks, "a range fits the staged record loads");
static_assert(kEntPad <= kEntOff, "entry offsets fit 13 bits");
constexpr int32_t kNodeFree = -1;       // bc_id of an unconstrained node
constexpr int32_t kNodePad = -2;        // bc_id of a padding node (never updated)

// Margin of the fast break decisions: a q (or a stretch) within this distance of a
// threshold t is decided on the exact stretch (stretch_exact).  The fast q carries a
// relative error near 1e-14 (one Newton step on the reciprocal length), the oracle's
// stretch an absolute error near 1e-16; the margin is far wider than both and so narrow
// that slots rarely land inside it.
__host__ __device__ inline double decision_margin(double t) { return 1e-9 * (t < 0.0 ? -t : t) + 1e-15; }

struct InstParams {
    double c;        // micromodulus without a stiffness field
    double q0;       // lower edge of the break decision on q = r^2/L^2 - 1: the threshold
                     // (1 + s0)^2 - 1 minus its margin (a slot at or above it takes the
                     // rare branch, which decides on the exact stretch); with damage laws,
                     // just below every law's elastic limit
    double s0;       // critical stretch of the brittle law
    double rho;
    double eta;
    double volume;   // uniform node volume without a volume array
    double bmag;     // body-force magnitude
    int32_t has_body;
    int32_t nlaw;    // damage laws of the instance (0: the brittle law with q0)
    int32_t law_off; // first law of the instance in StepArgs::laws
    int32_t pad_;
    double osb_a;    // state-based linear solid: 3K - 5G
    double osb_b;    // state-based linear solid: 15G
    // stiffness corrections evaluated per slot (kernels with CORR): flags bit 0 conical
    // profile 1 - |xi|/delta, bit 1 partial volume clamp((delta + dx/2 - |xi|)/dx, 0, 1),
    // bit 2 surface factor 2 V0 / (V_i + V_j) over family volumes
    double cr_idelta;  // 1/delta
    double cr_pvhi;    // (delta + dx/2)/dx
    double cr_idx;     // 1/dx
    double cr_2v0;     // 2 V0
    int32_t cr_flags;
    int32_t pad2_;
};

// Constraint of one node: per component d, kind in bits 2d..2d+1 (0 free, 1 displacement,
// 2 velocity) and schedule in bits 8+2d..9+2d (0 constant, 1 linear in t, 2 fifth-order
// ramp over T).
struct BCRec {
    double A[3];
    double T, iT;   // ramp duration and its reciprocal
    int32_t code;
    int32_t pad_;
};

// kModeForce evaluates the bond force density of the current level into StepArgs::force
// and changes nothing else (no integration, no breaking).
enum StepMode : int { kModeEC = 0, kModeVV = 1, kModeVVInit = 2, kModeFE = 3, kModeForce = 4 };

struct StepArgs {
    const double* rec_in;       // 6 doubles per node
    double* rec_out;
    double* v;                  // v + d*nn
    double* a;                  // a + d*nn
    const double* um_in;        // FP32 build: master displacement of the level read (d*nn + node)
    double* um_out;             // FP32 build: master displacement of the level written
    int32_t* col;
    const double* kslot;        // nullptr unless STIFF
    const double* vol;          // nullptr unless per-node volumes
    const double* na;           // nullptr unless per-node stiffness (then kslot is nullptr)
    const double* nw;
    const double* bhat;         // bhat + d*nn, nullptr without body forces
    double* force;              // kModeForce: bond force density out, force + d*nn
    const LawRec* laws;         // damage laws of every instance (nullptr without)
    const uint8_t* cls;         // per slot: law index within the instance (nullptr: 0)
    double* smax;               // per slot: largest stretch beyond the elastic limit
    double2* osb;               // state-based model: per node {theta / m, 1 / m} (nn + 128 entries)
    const double* minv;         // state-based model: per node 1 / m (padding 0)
    const double* cfv;          // corrections per slot: family volume per node (padding and the sentinel 1)
    const int64_t* slice_ptr;
    const int32_t* slice_T;
    const int32_t* slice_inst;
    const int32_t* slice_order; // staged step: slice of each workgroup in dispatch order (nullptr: its own)
    const InstParams* params;
    const int32_t* bc_id;
    const BCRec* bc;
    const int2* pieces;         // staged layout only
    const int32_t* slice_piece; // staged layout only
    uint16_t* ent;              // staged layout only
    const int64_t* step_base;   // completed steps when the launch sequence started
    int32_t* status;            // bit 0: a non-finite u or v was produced
    int32_t* bstep;             // per slot: the pass in which the slot broke (written on breaking)
    int64_t nn;                 // device node count (SoA stride); record nn is the sentinel
    int64_t nslices;
    int64_t step_local;         // this launch advances step *step_base + step_local
    double dt;
};

struct DamageArgs {
    const int32_t* col;
    int32_t sentinel;           // device index of the sentinel record (= node count)
    const double* vol;
    const int64_t* slice_ptr;
    const int32_t* slice_T;
    const int32_t* slice_inst;
    const InstParams* params;
    double* phi;
    int64_t nslices;
    const int2* pieces;         // staged layout only
    const int32_t* slice_piece;
    const uint16_t* ent;
    const LawRec* laws;         // damage laws (nullptr without)
    const uint8_t* cls;
    const double* smax;
};

// sliced mapping (FP64); ext: some slot may carry the no-failure bit or a damage law
// (the kernels with the bond-model branch)
hipError_t launch_step(const StepArgs& a, int lanes, int mode, bool stiff, bool ext, hipStream_t s);

// velocity-Verlet drift of every node (fp32: master displacement and f32 records)
hipError_t launch_drift(const StepArgs& a, bool fp32, hipStream_t s);

hipError_t launch_damage(const DamageArgs& a, int lanes, hipStream_t s);

// staged mapping, FP64 or FP32 bond arithmetic, `split` wavefronts per slice
hipError_t launch_step_staged(const StepArgs& a, int mode, bool fp32, int split, bool ext, hipStream_t s);
hipError_t launch_step_staged_f64(const StepArgs& a, int mode, int split, bool ext, hipStream_t s);
hipError_t launch_step_staged_f32(const StepArgs& a, int mode, int split, bool ext, hipStream_t s);

// out[d] = sum over the m device nodes idx[] of w_i field[i * snode + d * scomp], w_i = wv[i]
// or w when wv is nullptr, summed in a fixed order (force resultants, set means); with
// map, idx holds user node ids and node i is map[idx[r]]
hipError_t launch_set_sum(const double* field, int64_t snode, int64_t scomp, const double* wv, double w,
                          const int64_t* idx, int64_t m, double* out, hipStream_t s, const int64_t* map = nullptr);

// Allocation-free readouts: a per-GPU device array of kScratchNodes int64 node ids
// followed by 4 doubles, defined beside its kernels; its device address on `device`
// (looked up once per device, then cached; calls on one GPU share the array).
constexpr int64_t kScratchNodes = int64_t(1) << 18;
hipError_t scratch_address(int device, int64_t** out);

hipError_t launch_damage_staged(const DamageArgs& a, hipStream_t s);

// state-based linear solid (staged layout, FP64 or FP32 bond arithmetic): the dilation
// pass alone (breaking or a force evaluation), and a whole step (dilation pass, then the
// force pass with the integrator of `mode`)
hipError_t launch_osb_dilation(const StepArgs& a, bool breaking, bool fp32, int split, hipStream_t s);
hipError_t launch_osb_step(const StepArgs& a, int mode, bool fp32, int split, hipStream_t s);
constexpr int kOsbPad = 128;    // spare pairs after the last node (the pass-2 range copy)
constexpr int kCorrPad = 128;   // spare family volumes after the last node (the step kernels' copy window)

hipError_t launch_advance(int64_t* step_base, int64_t by, hipStream_t s);
// out[i * ncomp + d] = src[off + dnode[i] * snode + d * scomp], i < n (readout to device memory)
hipError_t launch_export_nodes(const double* src, int64_t snode, int64_t scomp, int64_t off, const int64_t* dnode,
                               int64_t n, int ncomp, double* out, hipStream_t s);
hipError_t launch_set_i64(int64_t* p, int64_t value, hipStream_t s);
// s[b] = the exact stretch (stretch_exact) of bond b, xi and y m x 3 row-major
hipError_t launch_stretch_exact(const double* xi, const double* y, double* s, int64_t m, hipStream_t st);

// ---------------------------------------------------------------- adjoint (Euler-Cromer)
//
// Break schedule per slot: bstep[ds] = pass in which the slot broke; kNeverBroke if it is
// intact, kBrokeBefore if it was broken before recording started (and for padding).  A
// slot acts in pass k iff k < bstep.
constexpr int32_t kNeverBroke = 0x7fffffff;
constexpr int32_t kBrokeBefore = -0x7fffffff - 1;

// One reverse pass k.  nu_in holds the adjoint of the unconstrained velocity of level
// k+1 (AoS, (nn+1) x 3, the last entry zero); lam_u (SoA) the adjoint of u^{k+1} on
// entry and of u^k on exit; nu_out receives the next pass's nu.
struct AdjArgs {
    const double* rec;          // node records (x, u^k), nn+1 of them
    const double* nu_in;
    double* nu_out;
    double* lam_u;
    double* grad;               // per device slot: d loss / d stiffness, accumulated
    double* gacc;               // per node: accumulated h * bhat . nu (body-force magnitude)
    const int32_t* bstep;
    const int32_t* col;         // sliced layout
    const uint16_t* ent;        // staged layout
    const int2* pieces;
    const int32_t* slice_piece;
    const double* kslot;
    const double* vol;
    const double* na;           // per-node stiffness factors sqrt(k_i) (or nullptr)
    const double* bhat;
    const int64_t* slice_ptr;
    const int32_t* slice_T;
    const int32_t* slice_inst;
    const InstParams* params;
    const int32_t* bc_id;
    const BCRec* bc;
    int64_t nn;
    int64_t nslices;
    int64_t k;                  // pass index
    double dt;
};

hipError_t launch_adjoint(const AdjArgs& a, bool staged, int lanes, hipStream_t s);
// bstep from the current broken flags: broken or padding -> kBrokeBefore, else kNeverBroke
hipError_t launch_bstep_init(int32_t* bstep, const int32_t* col, const uint16_t* ent, int64_t ns, hipStream_t s);
// broken flags as of level `step`: broken iff bstep < step
hipError_t launch_flags_at(const int32_t* bstep, int32_t* col, uint16_t* ent, int64_t ns, int64_t step, hipStream_t s);
// lam_u (SoA) += dL/du at the sensors, in order (repeated sensors add up)
hipError_t launch_adj_seed(double* lam_u, int64_t nn, const int64_t* sensors, const double* dldu, int64_t m,
                           hipStream_t s);
// nu = dt * lam_u on unconstrained components, 0 elsewhere (first reverse pass)
hipError_t launch_adj_nu0(double* nu, const double* lam_u, const int32_t* bc_id, const BCRec* bc, int64_t nn,
                          double dt, hipStream_t s);
// out[0] = sum of x[0..n)
hipError_t launch_sum(const double* x, int64_t n, double* out, hipStream_t s);

// lanes-per-node values with compiled kernels (sliced mapping)
bool lanes_supported(int lanes);
// wavefronts-per-slice values with compiled kernels (staged mapping)
bool split_supported(int split);

}  // namespace pdmi
