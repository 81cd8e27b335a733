/*
 * nbs.h -- C ABI of libnbs: two-baryon Nambu-Bethe-Salpeter four-point
 * functions by the effective baryon block algorithm, on AMD Instinct MI355X
 * (gfx950).
 *
 * The three compute calls follow the three stages of Eq. (6) of Nemura,
 * "An implementation of hybrid parallel CUDA code for the hyperonic nuclear
 * forces" (LATTICE 2015):
 *
 *   nbs_build_blocks       normal baryon blocks [B^(0)](x; xi1, xi2, xi3) of
 *                          Eq. (5) / Sec. 4(i) Eq. (8) on every sink site, then
 *                          their 3-D Fourier transform to momentum space
 *                          (Sec. 4(i));
 *   nbs_contract_channels  effective baryon blocks in momentum space
 *                          (Sec. 4(ii), Eq. (9)) and their products summed
 *                          over the shared source indices and diagrams
 *                          (Sec. 4(iii), Eq. (10)), giving F~_c(q) per channel;
 *   nbs_relative_sum       inverse Fourier transform with the 1/L^3 of
 *                          Eq. (6): the sum over X at every relative r, i.e.
 *                          F_c(r, t - t0) of Eq. (1).
 *
 * Every step runs in HIP kernels on the device; there is no host fallback.
 *
 * Conventions
 *   - Propagator of flavour f (u, d, s) on one time slice: 12 x 12 complex
 *     per site, row = 3 * spin + colour at the sink, column = 3 * spin +
 *     colour at the wall source.  Sites are ordered x + Lx * (y + Ly * z).
 *   - Spin components alpha_1..alpha_4 take the upper Dirac components
 *     {0, 1} (Dirac representation, C gamma_5 = diag(i s2, i s2)).
 *   - Output index s = 8 alpha_1 + 4 alpha_2 + 2 alpha_3 + alpha_4, and
 *     r = x_{B1} - x_{B2} mod L.
 *
 * Error behaviour: every call returns an nbs_status; nothing throws across
 * the ABI.  Arguments are validated on the host before any launch.  A HIP
 * failure maps to NBS_ERR_DEVICE and the message is kept per plan
 * (nbs_last_error).  A plan is not thread-safe; separate plans are
 * independent.
 */
#ifndef NBS_H
#define NBS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NBS_OK = 0,
  NBS_ERR_INVALID = 1,     /* bad argument (geometry, channel, pointer) */
  NBS_ERR_UNSUPPORTED = 2, /* valid request the library does not handle */
  NBS_ERR_NOMEM = 3,       /* device workspace does not fit */
  NBS_ERR_DEVICE = 4,      /* a HIP call failed */
  NBS_ERR_STATE = 5        /* calls out of order, or compute on a host-only plan */
} nbs_status;

typedef enum {
  NBS_FP64 = 0,     /* plain form: complex128 propagators, FP64 throughout */
  NBS_FP32_MFMA = 1 /* precision form: complex64 propagators and blocks
                       in storage, per-slice power-of-two scale, block
                       arithmetic in FP32, Fourier transforms computed in
                       FP64 (stored as complex64), effective blocks and
                       their products on the FP32 matrix cores
                       (v_mfma_f32_4x4x1f32, FP32 accumulation) with the
                       default launch shapes, FP64 channel normalisation.
                       The name says which matrix-core instruction the
                       contraction uses; it does not promise that every
                       step runs on matrix cores (the block build and the
                       transforms are vector-ALU code in both forms). */
} nbs_precision;

/* Interpolating fields of Eqs. (2)-(3). */
typedef enum {
  NBS_P = 0, NBS_N, NBS_LAMBDA, NBS_SIGMA_P, NBS_SIGMA_0, NBS_SIGMA_M,
  NBS_XI_0, NBS_XI_M, NBS_X_U, NBS_X_D, NBS_X_S, NBS_NUM_OPS
} nbs_op;

/* One lattice and one source slice.  The plan processes the window of
 * t_count consecutive sink slices starting at t_begin (absolute time);
 * t0 is the source slice.  L[0..2] = (Lx, Ly, Lz), each >= 2 and a product
 * of powers of 2, 3 and 5, at most 128. */
typedef struct {
  int32_t L[3];
  int32_t T, t0, t_begin, t_count;
} nbs_geometry;

/* Channel <B1 B2 | B3bar B4bar>: sink operators then source operators.
 * Flavour must be conserved (same u, d, s content on both sides). */
typedef struct {
  int32_t sink[2], src[2];
} nbs_channel;

typedef struct nbs_plan_s* nbs_plan;

/* Compile the channel table (Sec. 4(ii)-(iii): diagram classification into
 * structure-of-arrays tables, done once on the host) and allocate device
 * workspace.  g: n_geom geometries, 1 <= n_geom <= 32 (NBS_ERR_UNSUPPORTED
 * above).  Geometries may differ in every field (lattice extents, T, source
 * slice, window); each gets its own workspace, and the channel contraction
 * covers all of them in one launch (the batching form).
 * device >= 0: the HIP device to use; device == -1: host-only plan that
 * holds the compiled tables for inspection (nbs_plan_info, nbs_plan_diagrams,
 * nbs_plan_table, nbs_plan_params)
 * and rejects the compute calls with NBS_ERR_STATE.
 * On failure *out is NULL and nothing stays allocated. */
nbs_status nbs_plan_create(nbs_plan* out, const nbs_geometry* g, int32_t n_geom,
                           const nbs_channel* ch, int32_t n_ch,
                           nbs_precision prec, int32_t device);

/* Device bytes the plan owns (workspace + tables). */
nbs_status nbs_workspace_bytes(const nbs_plan plan, size_t* bytes);

/* Stage 1 (Eq. (5)/(8), then the forward transform of Eq. (6)).
 * prop_u/d/s[g]: device pointers, one per geometry, each
 * [t_count][Lz][Ly][Lx][12][12] complex (complex128 for NBS_FP64,
 * complex64 for NBS_FP32_MFMA), owned by the caller and read-only.
 * prop_d / prop_s may alias prop_u.  When prop_d[g] == prop_u[g] for every
 * geometry (the isospin-symmetric limit S_d = S_u of Sec. 4(i)), only the
 * canonical operator blocks are built and transformed and Sigma-, Xi- are
 * read as Sigma+, -Xi0 by the contraction (nbs_plan_table "op_alias",
 * "op_alias_coef"); n keeps its own block, since blocks are stored
 * antisymmetrised in their same-flavour slot pair and n's pair differs
 * from p's.  stream: a hipStream_t (NULL = the default
 * stream); the call is asynchronous on it. */
nbs_status nbs_build_blocks(nbs_plan plan, const void* const* prop_u,
                            const void* const* prop_d, const void* const* prop_s,
                            void* stream);

/* Stage 2 (Eqs. (9)-(10)): effective blocks and their products, F~_c(q).
 * Must follow nbs_build_blocks on the same plan. */
nbs_status nbs_contract_channels(nbs_plan plan, void* stream);

/* Stage 3 (inverse transform of Eq. (6), 1/L^3, undo of the per-slice
 * scale in FP64).  F_out[g]: device pointer, complex128
 * [n_ch][t_count][16][Lz][Ly][Lx], owned by the caller.  Must follow
 * nbs_contract_channels. */
nbs_status nbs_relative_sum(nbs_plan plan, void* const* F_out, void* stream);

/* A sink and a source operator of a single-baryon two-point function. */
typedef struct {
  int32_t sink, src;
} nbs_baryon_pair;

/* Zero-momentum single-baryon two-point functions, a by-product of stage 1:
 * Eq. (1) with one baryon at the sink and one at the (wall) source,
 *   C[a][a'](t) = sum_x sum over the source operator's flavour terms and the
 *   flavour-respecting Wick maps of the three source quarks, sign times the
 *   one-baryon source tensor eps (C g5) delta of Eq. (4) times the sink
 *   operator's normal block N(x)[a][...] of Eq. (5),
 * read from the transformed blocks at q = 0 (sum over x).  pairs: 1..8
 * (sink, src) operator codes; the sink operator must have a block in the
 * plan (a sink operator of one of its channels), else NBS_ERR_INVALID.
 * C_out[g]: device pointer, complex128 [n_pairs][t_count][2][2] (sink spin
 * a, source spin a'), owned by the caller.  Valid from nbs_build_blocks
 * until the next build (in either order with the other stages); undoes the
 * precision form's scale and, in the isospin-symmetric limit, reads n,
 * Sigma-, Xi- through their aliases.  Asynchronous on stream. */
nbs_status nbs_two_point(nbs_plan plan, const nbs_baryon_pair* pairs, int32_t n_pairs,
                         void* const* C_out, void* stream);

/* All three stages for every geometry as one captured HIP graph.  The first
 * call (and any call whose pointers differ from the captured ones) records
 * build, contract and relative sum into a graph on a plan-owned stream and
 * instantiates it; every call then launches the graph on `stream`.
 * Arguments as for the three stage calls; the plan is left as after
 * nbs_relative_sum.  The captured sequence contains no memset nodes. */
nbs_status nbs_run_graph(nbs_plan plan, const void* const* prop_u, const void* const* prop_d,
                         const void* const* prop_s, void* const* F_out, void* stream);

/* Measure launch-shape candidates on the device with the caller's
 * propagators and keep the fastest: for the block transforms, the one-pass
 * transform of 8^3 and 16^3 cubes, the fused x-y pass over square planes,
 * the register line kernel or LDS tiles of 512,
 * 1024, 2048 or 4096 elements; for the contraction, the matrix-core
 * segment engine with 8 or 16 wavefronts per workgroup or the lane-team
 * engine (8 wavefronts in FP64, 4 in the precision form), then the ranges
 * of sink-operator groups one workgroup walks, then (segment engine) a
 * workgroup per work item or resident workgroups claiming work items.  Synchronous; leaves the
 * plan as after nbs_build_blocks.  Results are unchanged up to rounding
 * order.  Callers that create the same shapes repeatedly can keep the
 * result (nbs_plan_tuning) and set it with nbs_plan_set_tuning instead. */
nbs_status nbs_plan_autotune(nbs_plan plan, const void* const* prop_u, const void* const* prop_d,
                             const void* const* prop_s, void* stream);

/* The plan's launch shapes: out[0] bit 0 register line FFT on/off, bit 1
 * fused x-y pass for square planes on/off, bit 2 one pass for all three
 * axes of 8^3 and 16^3 lattices on/off, forward and inverse (on by
 * default; the forward choices give the same blocks bit for bit, the
 * inverse ones the same F up to FP64 rounding order); out[1] LDS FFT tile
 * elements;
 * out[2] wavefronts per contraction workgroup of the selected engine;
 * out[3] bit 4 the contraction engine (1: matrix-core segments, the
 * default in both forms; 0: lane teams), bits 2-3 the contraction
 * workgroups per (slice, momentum): 0 one that walks every sink-operator
 * group, keeping an operator block in LDS while consecutive groups share
 * it; 1 one per run of groups in which one block stays; 2 one per group;
 * bit 5 (segment engine) persistent launch: as many workgroups as stay
 * resident, claiming (geometry, slice, momentum) work items from counters,
 * instead of one workgroup per item;
 * bits 0 and 1 apply to the lane-team engine only: bit 0 splitting a
 * product's walked index over lanes on/off, bit 1 (precision form) its
 * 4 x 4-row products on matrix cores on/off. */
nbs_status nbs_plan_tuning(const nbs_plan plan, int32_t out[4]);

/* Set the launch shapes (same encoding as nbs_plan_tuning) instead of
 * measuring them: waits for the plan's device work, recompiles the channel
 * program for the new shapes; blocks already built stay valid.  Rejects
 * (NBS_ERR_INVALID, the plan unchanged) unknown tiles, bits above bit 2 of
 * in[0] or bit 5 of in[3], wavefront counts other than 8 / 16 (segment engine) or 8 (lane
 * teams, FP64) or 4 / 8 (lane teams, precision form), matrix-core lane-team
 * products outside the precision form, group-range modes above 2 and the
 * persistent launch with the lane-team engine. */
nbs_status nbs_plan_set_tuning(nbs_plan plan, const int32_t in[4]);

/* Whether the propagators of the plan's last nbs_build_blocks (or
 * nbs_run_graph) held a NaN or an infinite entry: *found = 1 if so, else 0.
 * The block kernel checks every entry it reads; such entries are not
 * replaced, so the outputs of that build are not finite either, and in the
 * precision form an infinite maximum leaves the slice's scale at 1.  Waits
 * for all work on the plan's device.  NBS_ERR_STATE before the first build or
 * on a host-only plan. */
nbs_status nbs_plan_nonfinite(nbs_plan plan, int32_t* found);

/* Release everything the plan owns (waits for its device work). NULL is ok. */
nbs_status nbs_plan_destroy(nbs_plan plan);

const char* nbs_status_string(nbs_status s);
/* Message of the last failure on this plan ("" if none). */
const char* nbs_last_error(const nbs_plan plan);

/* ---- inspection of the compiled channel table (host-only) -------------- */

typedef struct {
  int32_t n_channels;
  int32_t n_types;        /* sink-operator blocks built (Lambda, Sigma0 from X_u, X_d, X_s) */
  int32_t n_diagrams;     /* (channel, source term, quark split) with both blocks non-empty */
  int32_t n_blocks;       /* distinct effective blocks (per momentum side) */
  int32_t n_products;     /* distinct block products after sharing across channels */
  int64_t sum_k;          /* sum over diagrams of |xi~_d| (shared-index count) */
  int64_t n_entries;      /* effective-block entries per momentum */
  int64_t n_terms;        /* normal-block reads per momentum to build them */
  int64_t n_wick_perms;   /* flavour-respecting Wick permutations covered */
} nbs_plan_info_t;

nbs_status nbs_plan_info(const nbs_plan plan, nbs_plan_info_t* info);

/* One diagram of one channel, in the paper's convention (Eq. (7)): the
 * source quarks given to the first sink baryon (bit k = source quark k+1),
 * the sign of the permutation that gives them in ascending order,
 * |xi~_d|, which of the labels alpha_3 / alpha_4 sit on the first block,
 * and the open (shared) source indices as a bit set over
 * (c'_k, alpha'_k): bit 2k = c'_{k+1}, bit 2k+1 = alpha'_{k+1}. */
typedef struct {
  int32_t channel, src_term, set1_mask, sign, k, labels1, open_mask;
  double coef;            /* full coefficient used (weights x sign) */
} nbs_diagram_t;

/* Copy up to cap diagrams of channel ch (ch = -1: all) into out; *n gets
 * the total count. */
nbs_status nbs_plan_diagrams(const nbs_plan plan, int32_t ch, nbs_diagram_t* out,
                             int32_t cap, int32_t* n);

/* Copy one table of the compiled structure-of-arrays program (the tables
 * the kernels interpret; Sec. 4(ii)-(iii) ship such tables to the device)
 * into buf.  int32 tables: "op_code", "op_nterm", "op_term_trip",
 * "op_term_perm", "op_pair" (s1 | s2 << 2 of the slot pair a block is
 * stored antisymmetrised and packed in, or -1), "op_alias", "group_op1",
 * "group_op2", "group_op1_iso", "group_op2_iso", "group_prod", "group_task",
 * "group_ch", "group_channels", "ch_contrib", "contrib_prod", "prod_desc",
 * "task_lanes", "seg_task", "group_stask", "prod_ext", "contrib_ext";
 * double tables: "contrib_coef", "op_term_w", "op_alias_coef",
 * "contrib_coef_iso".  *n gets the
 * element count; at most cap elements are written.  Unknown name:
 * NBS_ERR_INVALID.  Layouts are described in the compiler's header. */
nbs_status nbs_plan_table(const nbs_plan plan, const char* name, void* buf, int64_t cap, int64_t* n);

/* Program parameters: out[0] = ints per product descriptor, out[1] = lanes
 * per task, out[2] = most products in one group (LDS result buffer),
 * out[3] = most channels in one group. */
nbs_status nbs_plan_params(const nbs_plan plan, int32_t out[4]);

/* ---- without device allocation --------------------------------------- */

/* Device workspace (MiB) of nbs_four_point_static on each device. */
#define NBS_STATIC_WORKSPACE_MIB 64

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the whole
 * path of nbs_plan_create + nbs_build_blocks + nbs_contract_channels +
 * nbs_relative_sum for ONE geometry on the current device, with every
 * device buffer the path needs (operator blocks, F~, the compiled channel
 * program, the precision form's scales) carved from a workspace of
 * NBS_STATIC_WORKSPACE_MIB MiB that the library holds on each device it
 * runs on until the process ends; no hipMalloc or hipFree is called.
 * Arguments as for those calls: g one geometry, ch/n_ch the channels,
 * prop_u/d/s device pointers [t_count][Lz][Ly][Lx][12][12] (d may alias u:
 * the isospin limit), F_out device complex128 [n_ch][t_count][16][Lz][Ly][Lx].
 * The channel program is compiled on the host and uploaded on `stream`
 * (this call waits for the upload), the kernels are enqueued on `stream`.
 * Errors: NBS_ERR_UNSUPPORTED when the problem needs more device memory than
 * the workspace (nbs_static_last_error gives the size), otherwise as
 * nbs_plan_create and the stage calls.  Every call on a device shares that
 * device's workspace and overwrites what the previous call left there:
 * calls that overlap on one device (different streams or host threads)
 * race; calls on one stream are ordered.  Results equal those of the plan
 * path with default launch shapes. */
nbs_status nbs_four_point_static(const nbs_geometry* g, const nbs_channel* ch, int32_t n_ch,
                                 nbs_precision precision, const void* prop_u, const void* prop_d,
                                 const void* prop_s, void* F_out, void* stream);

/* Message of the last failed nbs_four_point_static call ("" if none). */
const char* nbs_static_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* NBS_H */
