/*
 * mpdp.h -- C-ABI of the MI355X (gfx950) MPDP join-order optimizer.
 *
 * MPDP (arXiv 2202.13511) finds the cheapest cross-product-free bushy join
 * tree of a query by a dynamic program over connected relation subsets,
 * level by level in subset size (Section 5, Alg. 5): for every size k it
 * unranks the k-subsets, filters the connected ones, enumerates their valid
 * join pairs (csg-cmp pairs, Section 2.1) with the block-based enumeration of
 * Section 3.2 (Alg. 3; Alg. 2 when the join graph is a tree), costs every
 * pair, keeps the best pair per subset and writes it to the memo.  All of
 * that runs as HIP kernels on one GPU; the host only validates the input,
 * uploads a few kilobytes of query information and reads back the plan.
 *
 * Query information (QI of Alg. 1 / Alg. 5): relations 0..n-1, one edge per
 * join predicate, base cardinalities and edge selectivities.
 *
 * Shared definitions (the paper leaves estimation and cost formulas open,
 * Section 7.1; these are this library's):
 *   card(S)  c = 1.0; for v in S ascending { c = c*card[v]; for u in S,
 *            u < v, (u,v) an edge, ascending: c = c*sel(u,v) };
 *            card(S) = (c < 1.0) ? 1.0 : c.  Evaluated in IEEE binary64,
 *            left to right, no fused multiply-add.
 *   C_out    cost({v}) = 0; cost(L join R) = (cost(L) + cost(R)) + card(L u R).
 *   PG-like  cost({v}) = 0.01*card[v];
 *            HJ = (((cL + cR) + 0.0125*card(R)) + 0.0025*card(L)) + 0.01*card(S)
 *            NL = ((cL + cR) + (0.0025*card(L))*card(R)) + 0.01*card(S)
 *            (PostgreSQL's default cpu_tuple_cost 0.01 and
 *            cpu_operator_cost 0.0025; R is the hashed / inner side).
 *   Best plan of S: the smallest key (cost, left relation bitmap, op) over
 *            all candidates, with HASH < NESTLOOP.  The result is independent
 *            of enumeration order and launch configuration.
 *
 * Bitmaps: bit v of a uint32_t stands for relation v (n <= 32).
 */
#ifndef MPDP_H
#define MPDP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MPDP_OK = 0,
    MPDP_EINVAL = 1,         /* malformed input or null required pointer           */
    MPDP_ENOTCONNECTED = 2,  /* join graph disconnected: no cross-product-free plan */
    MPDP_ETOOLARGE = 3,      /* n > 32: beyond the bitmap width of the exact DP    */
    MPDP_ENOMEM = 4,         /* workspace too small, or device allocation failed   */
    MPDP_EDEVICE = 5,        /* a HIP runtime error                                */
    MPDP_ETIMEOUT = 6        /* budgeted heuristics: the time budget ran out; the
                                outputs hold the complete plan found so far       */
} mpdp_status;

typedef enum { MPDP_COST_COUT = 0, MPDP_COST_PGLIKE = 1 } mpdp_cost_model;

typedef enum {
    MPDP_OP_SCAN = 0,      /* base relation                         */
    MPDP_OP_HASH = 1,      /* hash join (PG-like)                   */
    MPDP_OP_NESTLOOP = 2,  /* nested-loop join (PG-like)            */
    MPDP_OP_JOIN = 3       /* logical join (C_out has no operator)  */
} mpdp_op;

/* One join predicate between relations u and v (0-based, u != v). */
typedef struct { uint32_t u, v; } mpdp_edge;

/* One node of the plan tree (Section 5: the best plan is rebuilt from the
 * memo by following left/right).  plan_out holds 2n-1 nodes: nodes 0..n-1 are
 * the base relations in index order, join nodes follow in post-order (left
 * subtree, right subtree, node) and the root is node 2n-2. */
typedef struct {
    int32_t left, right;   /* child node index, -1 for a base relation     */
    uint32_t relset;       /* relations under this node                     */
    uint32_t op;           /* mpdp_op                                       */
    double cost;           /* cost of the subplan                           */
    double card;           /* card(relset)                                  */
} mpdp_plan_node;

/* Counters (Section 2.1 / Alg. 1 counters, with explicit conventions). */
typedef struct {
    uint64_t candidates;       /* subsets unranked: sum over k >= 2 of C(n,k)                 */
    uint64_t connected_sets;   /* connected subsets with >= 2 relations                       */
    uint64_t evaluated_pairs;  /* Alg. 3 EvaluatedCounter: sum over sets and blocks of 2^b - 2 */
    uint64_t ccp_pairs;        /* csg-cmp pairs, unordered ((L,R) and (R,L) count once)        */
    double ms_total;           /* host wall time of the call                                  */
    double ms_filter;          /* device time of the unrank/filter kernels (MPDP_FLAG_TIMING) */
    double ms_eval;            /* device time of the evaluate kernels      (MPDP_FLAG_TIMING) */
    uint32_t levels;           /* number of DP levels run (n - 1)                             */
    uint32_t eval_launches;    /* evaluate-kernel launches                                    */
} mpdp_stats;

/* Flags for mpdp_optimize_ws. */
#define MPDP_FLAG_TIMING 1u   /* time the filter and evaluate kernels with HIP events */
/* Ablations (measurement only; plans, costs and ccp counts are unchanged):
 * DPSUB      every connected set takes DPSUB's vertex-based candidates (Alg. 1:
 *            every subset holding its lowest relation, CCP-checked) instead of
 *            Alg. 2/3's block-local ones; evaluated_pairs counts 2^|S| - 2 per set
 * NO_COMPACTION  tree joins: each lane evaluates the connected candidates it
 *            unranked instead of compacting them through the wave's LDS ring;
 *            a tree of depth one from relation 0 (a star around it), whose
 *            connected sets are otherwise enumerated directly, is then
 *            unranked and filtered over every k-subset as well
 * UNFUSED_PRUNE  tree joins: prune is not fused into evaluate (Section 5,
 *            "Enhancements"): the evaluate kernel writes the key of every
 *            pair to global memory and a separate prune kernel reduces each
 *            set's keys and writes its memo entry; the library allocates the
 *            key buffer (16 bytes per pair of the widest level) once per
 *            device and keeps it */
#define MPDP_FLAG_ABLATE_DPSUB 2u
#define MPDP_FLAG_ABLATE_NO_COMPACTION 4u
#define MPDP_FLAG_ABLATE_UNFUSED_PRUNE 8u

/* Status string for an mpdp_status value (static storage, never NULL). */
const char *mpdp_status_str(mpdp_status s);

/* Bytes of device workspace mpdp_optimize_ws needs for n relations
 * (0 if n is 0 or above 32): a memo entry of 21 bytes for every subset of
 * the relations (2^n entries) plus one level of candidate sets. */
size_t mpdp_workspace_bytes(uint32_t n, mpdp_cost_model cost_model);

/* Byte offsets of the memo arrays inside the workspace, for callers that
 * inspect the memo after a successful call: cost (double[2^n]), card
 * (double[2^n]), left (uint32_t[2^n]: left input relation set of the best
 * join, 0 for base relations), op (uint8_t[2^n]).  The memo is
 * level-compact: the entry of relation set S is at index
 *     off(|S|) + colex(S),  off(k) = sum_{j<k} C(n, j),
 *     colex(S) = sum over the members s_0 < s_1 < ... of C(s_i, i + 1),
 * so each DP level is one contiguous slab.  Only entries of connected sets
 * are defined.  Returns MPDP_EINVAL for n outside 1..32 or a null pointer. */
mpdp_status mpdp_memo_layout(uint32_t n, size_t *off_cost, size_t *off_card, size_t *off_left,
                             size_t *off_op);

/*
 * Optimize one query on the current HIP device.
 *   n, m          relations and edges (m may be 0 only when n == 1)
 *   edges         host, m entries; no self loops, no duplicate pairs
 *   cardinalities host, n finite values >= 1
 *   selectivities host, m finite values in (0, 1], one per edge
 *   cost_model    MPDP_COST_COUT or MPDP_COST_PGLIKE
 *   plan_out      host, caller-allocated, 2n-1 nodes (layout above)
 *   cost_out      host, receives the root cost
 *   stats_out     host, optional (NULL to skip)
 * The library allocates and frees its own workspace and uses the null
 * stream; it keeps no pointer after returning.  Outputs are written only on
 * MPDP_OK.  Validation happens on the host before any HIP call, so every
 * error except MPDP_ENOMEM / MPDP_EDEVICE is reported without a GPU.
 */
mpdp_status mpdp_optimize(uint32_t n, uint32_t m, const mpdp_edge *edges,
                          const double *cardinalities, const double *selectivities,
                          mpdp_cost_model cost_model, mpdp_plan_node *plan_out,
                          double *cost_out, mpdp_stats *stats_out);

/*
 * As mpdp_optimize, with caller-owned device memory and stream:
 *   d_workspace   device pointer to at least mpdp_workspace_bytes(n, cost_model)
 *                 bytes, 256-byte aligned; contents on entry are ignored
 *   ws_bytes      its size (MPDP_ENOMEM if too small)
 *   hip_stream    hipStream_t to enqueue on (NULL: the null stream)
 *   flags         0, or MPDP_FLAG_TIMING and the ablation flags
 * All kernels run on hip_stream; the call waits for that stream before it
 * returns because the plan is delivered to host memory.  Concurrent calls
 * must use distinct workspaces.  After MPDP_OK the memo stays readable in the
 * workspace (mpdp_memo_layout).
 */
mpdp_status mpdp_optimize_ws(uint32_t n, uint32_t m, const mpdp_edge *edges,
                             const double *cardinalities, const double *selectivities,
                             mpdp_cost_model cost_model, void *d_workspace, size_t ws_bytes,
                             void *hip_stream, uint32_t flags, mpdp_plan_node *plan_out,
                             double *cost_out, mpdp_stats *stats_out);

/* Largest query mpdp_optimize_noalloc takes. */
#define MPDP_NOALLOC_MAX_REL 20u

/*
 * For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): mpdp_optimize_ws with the
 * workspace replaced by a fixed device array inside the library.
 *   n             at most MPDP_NOALLOC_MAX_REL; MPDP_ETOOLARGE beyond
 *   hip_stream    hipStream_t to enqueue on (NULL: the null stream)
 *   flags         0 or the ablation flags; MPDP_FLAG_TIMING is MPDP_EINVAL
 *   other arguments, outputs and validation as in mpdp_optimize_ws
 * The call allocates nothing, on the host or the device: the array
 * (mpdp_noalloc_scratch_bytes() bytes, 24 MiB) exists on every device the
 * library runs on and is held until the process ends; its device address is
 * looked up on the first call on each device.  The query information goes up
 * and the plan comes back through pageable copies from the caller's thread.
 * Every call on one device uses that device's one array, so calls that
 * overlap on one device (from several threads or streams) race and must be
 * serialised by the caller; each call rewrites everything it reads, so no
 * state carries over from the previous call.  The call waits for its stream.
 */
size_t mpdp_noalloc_scratch_bytes(void);
mpdp_status mpdp_optimize_noalloc(uint32_t n, uint32_t m, const mpdp_edge *edges,
                                  const double *cardinalities, const double *selectivities,
                                  mpdp_cost_model cost_model, void *hip_stream, uint32_t flags,
                                  mpdp_plan_node *plan_out, double *cost_out, mpdp_stats *stats_out);

/*
 * As mpdp_optimize_ws for a query whose relations stand for intermediate
 * results that are already planned (the exact step of IDP2 and UnionDP,
 * Section 4: "temporary tables" and composite nodes): relation v costs
 * base_costs[v] (host, n values, finite, >= 0) instead of its scan; its
 * cardinality is cardinalities[v] as usual.  Everything else, including the
 * workspace size, is as in mpdp_optimize_ws.  MPDP_EINVAL if base_costs is
 * NULL or holds a negative or non-finite value.
 */
mpdp_status mpdp_optimize_units(uint32_t n, uint32_t m, const mpdp_edge *edges,
                                const double *cardinalities, const double *selectivities,
                                const double *base_costs, mpdp_cost_model cost_model,
                                void *d_workspace, size_t ws_bytes, void *hip_stream, uint32_t flags,
                                mpdp_plan_node *plan_out, double *cost_out, mpdp_stats *stats_out);

/*
 * The same exact DP on the host's cores (the all-cores CPU baseline of the
 * measurements; Section 3.3 hands out work items through an atomic
 * counter): every level's colex rank range is cut into chunks that
 * `threads` threads (0: all hardware threads) take from an atomic counter;
 * enumeration, card(S), costs and the plan key are those above, so the
 * plan and cost equal the GPU's bit for bit.  Dense memo of 2^n entries in
 * host memory; n <= 28 (MPDP_ETOOLARGE beyond); no HIP call.  Arguments and
 * errors otherwise as mpdp_optimize; stats_out->eval_launches holds the
 * thread count.
 */
mpdp_status mpdp_optimize_cpu(uint32_t n, uint32_t m, const mpdp_edge *edges,
                              const double *cardinalities, const double *selectivities,
                              mpdp_cost_model cost_model, uint32_t threads, mpdp_plan_node *plan_out,
                              double *cost_out, mpdp_stats *stats_out);

/*
 * Batched optimization: many small queries in one launch.
 *
 * Query q has n relations whose cardinalities are
 * cardinalities[card_offset .. card_offset + n) and m edges whose endpoints
 * (0-based within the query) and selectivities are
 * edges/selectivities[edge_offset .. edge_offset + m).  Every query obeys
 * the rules of mpdp_optimize and has 1 <= n <= 20.
 */
typedef struct { uint32_t n, m, card_offset, edge_offset; } mpdp_batch_query;

typedef struct {
    uint64_t connected_sets;   /* summed over the batch (conventions as mpdp_stats) */
    uint64_t evaluated_pairs;
    uint64_t ccp_pairs;
    double ms_total;           /* host wall time of the call                            */
    double ms_kernel;          /* device time of the batch kernel (MPDP_FLAG_TIMING)      */
    uint32_t workgroups;       /* persistent workgroups launched                        */
    uint32_t max_n;            /* largest query in the batch                            */
} mpdp_batch_stats;

/* Device workspace bytes for mpdp_optimize_batch (0 if a query is invalid in
 * size: n = 0 or n > 20).  It grows with the total input and output sizes
 * and with at most 512 memo slots of 2^max_n entries, not with nq itself
 * (plus a few hundred bytes per cyclic query of 17 or more relations, which
 * may be shared by a team of workgroups). */
size_t mpdp_batch_workspace_bytes(uint32_t nq, const mpdp_batch_query *queries);

/*
 * Optimize nq queries in one persistent launch on hip_stream: every
 * workgroup takes the next query, runs all its DP levels with workgroup
 * barriers between levels, and writes its plan.  A cyclic query of 17 or
 * more relations that is predicted to be slow is taken by a team of 4 or 8
 * workgroups, which split every level and meet at device-wide barriers
 * (each wait bounded; a team that times out reports MPDP_EDEVICE).
 * Results equal those of mpdp_optimize on each query alone.
 *   plans_out      host, sum over q of (2 n_q - 1) nodes; query q's plan
 *                  (layout of mpdp_plan_node) starts after those of 0..q-1
 *   costs_out      host, nq root costs
 *   latency_us_out host, nullable: per query, microseconds from the start of
 *                  the launch to the end of that query (device wall clock)
 *   start_us_out   host, nullable: per query, microseconds from the start of
 *                  the launch to the start of that query
 *   stats_out      host, nullable
 * Workgroups take the queries in order of decreasing predicted time (from
 * the query's shape: its relations, extra edges, the connected subsets of a
 * spanning tree and the size of its 2-core; ties in input order), which
 * shortens the tail of the launch.
 * Validation is done on the host before any HIP call (MPDP_EINVAL,
 * MPDP_ENOTCONNECTED, MPDP_ETOOLARGE name the first failing query's error);
 * the call waits for hip_stream before returning.
 */
mpdp_status mpdp_optimize_batch(uint32_t nq, const mpdp_batch_query *queries, const mpdp_edge *edges,
                                const double *cardinalities, const double *selectivities,
                                mpdp_cost_model cost_model, void *d_workspace, size_t ws_bytes,
                                void *hip_stream, uint32_t flags, mpdp_plan_node *plans_out,
                                double *costs_out, double *latency_us_out, double *start_us_out,
                                mpdp_batch_stats *stats_out);

/*
 * Schedule of one query in the batched kernel (defaults in brackets, which
 * mpdp_optimize_batch uses):
 *   tree_chunk    acyclic queries: consecutive colex ranks per lane in each
 *                 level's fused unrank, filter and evaluate pass: 1, 2 or 4 [4]
 *   heavy_chunks  cyclic queries: a set whose Alg. 3 candidates fill more
 *                 than this many chunks of 16 is evaluated by the whole
 *                 workgroup, a smaller one by one wave: 1 .. 65535 [256]
 * Every schedule gives the same plans and costs; only the time differs.
 */
typedef struct { uint32_t tree_chunk, heavy_chunks; } mpdp_batch_schedule;

/* mpdp_optimize_batch with a schedule per query: schedules is host memory,
 * nq entries in input order, or NULL for the defaults.  MPDP_EINVAL for a
 * schedule outside the ranges above; everything else as mpdp_optimize_batch. */
mpdp_status mpdp_optimize_batch_sched(uint32_t nq, const mpdp_batch_query *queries, const mpdp_edge *edges,
                                      const double *cardinalities, const double *selectivities,
                                      mpdp_cost_model cost_model, void *d_workspace, size_t ws_bytes,
                                      void *hip_stream, uint32_t flags, const mpdp_batch_schedule *schedules,
                                      mpdp_plan_node *plans_out, double *costs_out, double *latency_us_out,
                                      double *start_us_out, mpdp_batch_stats *stats_out);

typedef struct {
    uint32_t classes;       /* query classes tuned                                        */
    uint32_t launches;      /* batch launches spent timing candidates                      */
    double ms_total;        /* host wall time of the tuning                                */
    double est_default_ms;  /* sum over queries of their class's median device time, defaults */
    double est_tuned_ms;    /* the same with the chosen schedules                          */
} mpdp_batch_tune_stats;

/*
 * Autotuner of the batched kernel's per-query schedule.  Queries fall into
 * classes by (n, whether the join graph is a tree, edges beyond a spanning
 * tree: 0, 1-2, 3-5, 6 or more).  Each candidate (tree_chunk 1, 2, 4;
 * heavy_chunks 32, 64, 128, 256, 1024) runs over the whole batch `reps`
 * times, acyclic and cyclic candidates sharing launches; every query's
 * device time comes from the kernel's clock at its start and end, and each
 * class gets the candidate with the smallest median time over its queries
 * and repetitions (ties to the default).  schedules_out: host, nq entries in
 * input order.  reps in 1..16; other arguments and errors as in
 * mpdp_optimize_batch (the workspace is sized by mpdp_batch_workspace_bytes).
 */
mpdp_status mpdp_batch_autotune(uint32_t nq, const mpdp_batch_query *queries, const mpdp_edge *edges,
                                const double *cardinalities, const double *selectivities,
                                mpdp_cost_model cost_model, void *d_workspace, size_t ws_bytes, void *hip_stream,
                                uint32_t reps, mpdp_batch_schedule *schedules_out,
                                mpdp_batch_tune_stats *stats_out);

/*
 * A batch captured in a HIP graph: the upload of the query data, the
 * persistent batched kernel and the downloads of plans, costs and clocks are
 * recorded once for a fixed batch shape (every query's n and m, the cost
 * model, the workspace) and replayed with new data by mpdp_batch_graph_run,
 * so a serving loop issues one graph launch per batch.  The handle owns
 * pinned host staging buffers (hipHostMalloc).  The workspace, sized by
 * mpdp_batch_workspace_bytes, must outlive the handle and not be used by
 * other calls meanwhile; replays of one handle must not overlap.
 * mpdp_batch_graph_create returns MPDP_EINVAL for a bad shape or workspace
 * and MPDP_EDEVICE if capture fails; *graph_out is NULL on error.
 */
typedef struct mpdp_batch_graph mpdp_batch_graph;

mpdp_status mpdp_batch_graph_create(uint32_t nq, const mpdp_batch_query *queries, mpdp_cost_model cost_model,
                                    void *d_workspace, size_t ws_bytes, mpdp_batch_graph **graph_out);

/* One replay on hip_stream, waited for.  queries must have, query by query,
 * the n and m given at creation (their offsets may differ); the data are
 * validated as in mpdp_optimize_batch; schedules as in
 * mpdp_optimize_batch_sched; outputs as in mpdp_optimize_batch. */
mpdp_status mpdp_batch_graph_run(mpdp_batch_graph *graph, const mpdp_batch_query *queries,
                                 const mpdp_edge *edges, const double *cardinalities,
                                 const double *selectivities, const mpdp_batch_schedule *schedules,
                                 void *hip_stream, mpdp_plan_node *plans_out, double *costs_out,
                                 double *latency_us_out, mpdp_batch_stats *stats_out);

/* Free the handle, its graph and its staging buffers (NULL is ignored). */
void mpdp_batch_graph_destroy(mpdp_batch_graph *graph);

/*
 * Large queries (Section 4): heuristics that hand sub-problems of at most k
 * units to the exact DP above, on the GPU.
 *   MPDP_LARGE_GOO      greedy operator ordering alone: join the two
 *                       connected trees whose union has the smallest card
 *   MPDP_LARGE_IDP2     IDP2 (Section 4.1) with GOO's plan as the start:
 *                       repeatedly re-plan, exactly, the costliest subtree of
 *                       2..k units and make it one unit
 *   MPDP_LARGE_UNIONDP  UnionDP (Section 4.2, Alg. 4): partition the graph of
 *                       units into connected parts of at most k units (union
 *                       order: size of the two parts, then the card of the
 *                       edge's two units), plan each part exactly (all parts
 *                       of one round in one batched launch when they have at
 *                       most 20 units), and repeat on the graph of parts
 * A unit reaches the exact step as one relation: card(S) of its relation
 * set, its plan's cost as base cost, and one edge to each adjacent unit
 * whose selectivity is the product of the base selectivities between them
 * (edge-list order; clamped below at the smallest normal double).  Every
 * plan is finally re-costed over the base relations: card(S) as defined at
 * the top of this header for any relation set, each join in its cheaper
 * orientation and operator (key: cost, then the left relation set read as a
 * binary number, then HASH before NESTLOOP).  cost_out is that cost.
 */
typedef enum {
    MPDP_LARGE_GOO = 0,
    MPDP_LARGE_IDP2 = 1,
    MPDP_LARGE_UNIONDP = 2,
    MPDP_LARGE_UNIONDP_LEARNED = 3  /* UnionDP whose partition phase is driven by the scorer of
                                       mpdp_scorer.h (not part of the paper): parts start as single
                                       units; each pass scores every union of two adjacent parts with
                                       at most k units together and joins the best-scored one (ties by
                                       part pair order) if its logit is positive; passes repeat until
                                       none joins.  A round whose first pass joins nothing falls back to
                                       the paper's order (plain UnionDP). */
} mpdp_large_method;

/* Plan node of a large query.  Nodes 0..n-1 are the relations in index
 * order; join nodes follow in post-order (left child first); the root is
 * node 2n-2. */
typedef struct {
    int32_t left, right;  /* child node indices, -1 for leaves                 */
    uint32_t rel;         /* leaf: its relation; join: lowest relation below it */
    uint32_t nrels;       /* relations below this node                        */
    uint32_t op, pad;     /* mpdp_op                                          */
    double cost, card;
} mpdp_large_node;

typedef struct {
    uint64_t exact_calls;  /* sub-problems planned by the exact DP              */
    uint64_t exact_units;  /* units over all exact sub-problems                 */
    uint32_t max_units;    /* largest exact sub-problem                         */
    uint32_t rounds;       /* IDP2 iterations or UnionDP partition rounds       */
    uint32_t launches;     /* exact-step calls into the GPU (a batch counts 1)  */
    uint32_t pad;
    double ms_total;       /* host wall time of the call                        */
    double ms_exact;       /* of which in the exact step (upload, kernels, readback) */
} mpdp_large_stats;

/*
 * Plan a query of 1 <= n <= 4096 relations with `method` and sub-problem
 * bound 2 <= k <= 25 (ignored by GOO).  d_scorer is a device parameter
 * block of mpdp_scorer.h (required by MPDP_LARGE_UNIONDP_LEARNED, ignored
 * otherwise; the features of a candidate union are listed at
 * mpdp_large_examples).  Inputs follow mpdp_optimize (edges
 * with distinct unordered endpoint pairs, card >= 1 finite, sel in (0, 1],
 * connected join graph), except for the bound on n.
 *   plan_out   host, caller-allocated, 2n-1 nodes (layout above)
 *   cost_out   host, the plan's re-costed cost
 *   stats_out  host, optional
 * The library allocates its device workspace (for k units, or for a round of
 * batched parts) and frees it before returning; it runs on hip_stream (NULL:
 * the null stream).  MPDP_EINVAL for malformed input, k out of range or an
 * unknown method; MPDP_ENOTCONNECTED; MPDP_ETOOLARGE for n > 4096;
 * MPDP_ENOMEM / MPDP_EDEVICE from the device.  Outputs are written only on
 * MPDP_OK.
 */
mpdp_status mpdp_optimize_large(uint32_t n, uint32_t m, const mpdp_edge *edges,
                                const double *cardinalities, const double *selectivities,
                                mpdp_cost_model cost_model, mpdp_large_method method, uint32_t k,
                                const void *d_scorer, void *hip_stream, mpdp_large_node *plan_out,
                                double *cost_out, mpdp_large_stats *stats_out);

/*
 * mpdp_optimize_large with a wall-clock budget (Section 4.1: IDP2 can stop
 * whenever a budget is exhausted), budget_ms > 0 counted from the call's
 * start (0: none; negative or non-finite: MPDP_EINVAL).  The budget is
 * checked before every exact sub-problem and every scored pass of the
 * learned partition; a sub-problem already started runs to its end.  When
 * it has run out, the call returns MPDP_ETIMEOUT with plan_out, cost_out and
 * stats_out written:
 *   IDP2     the GOO start with the subtrees re-planned so far (every
 *            re-planning only lowers the cost, so this is never worse than
 *            GOO alone);
 *   UnionDP  (plain or learned) the units of the current round, each with
 *            its exact plan, joined by GOO (smallest union card first);
 *   GOO      ignores the budget.
 */
mpdp_status mpdp_optimize_large_budget(uint32_t n, uint32_t m, const mpdp_edge *edges,
                                       const double *cardinalities, const double *selectivities,
                                       mpdp_cost_model cost_model, mpdp_large_method method, uint32_t k,
                                       const void *d_scorer, double budget_ms, void *hip_stream,
                                       mpdp_large_node *plan_out, double *cost_out,
                                       mpdp_large_stats *stats_out);

/*
 * Training examples for the scorer from a query of n <= 32 relations whose
 * optimal plan is known (plan_sets: the relation bitmaps of its nsets
 * nodes): run learned UnionDP with bound k, driven by d_scorer, or, with
 * d_scorer NULL, by the teacher that scores a union +1 when it is a node of
 * the optimal plan and -1 otherwise; emit one row per candidate union of
 * every pass: MPDP_SCORER_IN BF16 features and a label, 1 iff the union is a
 * node of the optimal plan.
 * Features of the union of parts A and B (parts numbered by their lowest
 * unit, pairs ascending), w = card(A u B), each pair put as (smaller,
 * larger), computed in binary64 and rounded to binary32 and then to BF16
 * (nearest even): 0,1 log10 card(A), card(B) / 8; 2 log10 w / 8;
 * 3 (log10 w - log10 card(A) - log10 card(B)) / 8; 4,5 log10(1 + summed plan
 * cost of the units of A, B) / 8; 6,7 log2 of their relation counts / 4;
 * 8,9 their numbers of candidate unions / 8; 10,11 their unit counts / 8;
 * 12,13 the share of A's (B's) candidates with a smaller weight than w;
 * 14,15 log10 w - log10 of the smallest weight of a candidate of A (B), / 8;
 * 16 log2 of the parts / 12; 17 the share of all candidates with a smaller
 * weight; 18 one; 19..31 zero.
 * features_out (host, max_examples x MPDP_SCORER_IN), labels_out (host,
 * max_examples), count_out (host): the number of rows; MPDP_ENOMEM (with
 * count_out set) when it exceeds max_examples.
 */
mpdp_status mpdp_large_examples(uint32_t n, uint32_t m, const mpdp_edge *edges,
                                const double *cardinalities, const double *selectivities,
                                mpdp_cost_model cost_model, uint32_t k, const void *d_scorer,
                                const uint32_t *plan_sets, uint32_t nsets, void *hip_stream,
                                uint16_t *features_out, float *labels_out, uint32_t max_examples,
                                uint32_t *count_out);

#ifdef __cplusplus
}
#endif

#endif /* MPDP_H */
