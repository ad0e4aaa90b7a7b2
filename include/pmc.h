/*
 * pmc.h - C ABI of the progressive material cache library (libpmc.so).
 *
 * The library shades batches of ray hits with node-based material networks
 * on one MI355X (gfx950).  Selected node outputs are looked up in, and
 * progressively inserted into, a fixed-size device hash table keyed by
 * material id, node id and a quantised UV texel, using two hashes: one picks
 * the cell, the other verifies the key (Fujieda & Harada, "Progressive
 * Material Caching", SIGGRAPH Asia 2022 TC: Sec. 2 network evaluation,
 * Sec. 3 cacheable nodes, Sec. 3.1 descriptor and Eq. 1, Sec. 3.2 the two
 * hashes, Sec. 3.3 and Algorithm 1 the lock-free update).
 *
 * Conventions for every entry point
 *   - Return value: PMC_OK (0) or a negative pmc_status.  Nothing throws
 *     across this boundary.  pmc_last_error() gives the message of the last
 *     failing call on a context.
 *   - Argument and graph errors are detected on the host before any work is
 *     enqueued; nothing is enqueued when a call fails.
 *   - Data errors inside a batch never abort: a material id at or beyond the
 *     compiled count shades to default outputs and is counted; non-finite
 *     UVs or gradients bypass the cache.
 *   - Pointers named "device" are device memory (e.g. from hipMalloc or a
 *     torch CUDA tensor) owned by the caller; "host" pointers are read (or
 *     written) before the call returns, unless the entry point says it runs
 *     asynchronously on the stream.
 *   - Streams are passed as void* (a hipStream_t; NULL = the null stream).
 *     Device work is enqueued on that stream only; calls return without
 *     waiting unless stated.
 *   - A context is not thread-safe.  Different contexts are independent.
 */
#ifndef PMC_H
#define PMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PMC_ABI_VERSION 6u

typedef int32_t pmc_status;
enum {
    PMC_OK = 0,
    PMC_ERR_INVALID = -1,      /* bad argument (null pointer, size, enum value) */
    PMC_ERR_GRAPH = -2,        /* invalid material network (type, cycle, link) */
    PMC_ERR_OOM = -3,          /* device or host allocation failed */
    PMC_ERR_HIP = -4,          /* a HIP runtime call failed; message has hipGetErrorString */
    PMC_ERR_UNSUPPORTED = -5,  /* valid request the library cannot serve */
    PMC_ERR_STATE = -6         /* call order (e.g. shading before compiling) */
};

typedef struct pmc_ctx pmc_ctx;        /* opaque, library-owned */
typedef struct pmc_cache pmc_cache;    /* opaque handle of one hash table */

/* ------------------------------------------------------------------ graphs */

/* Node operations (Sec. 2 leaves node types open; this is the library's set). */
enum pmc_op {
    PMC_OP_UV_INPUT = 0,       /* out 0: UV of the hit */
    PMC_OP_IMAGE_TEXTURE = 1,  /* in 0: UV; out 0: COLOR, out 1: FLOAT alpha */
    PMC_OP_VALUE_NOISE = 2,    /* in 0: UV; out 0: FLOAT */
    PMC_OP_PERLIN_NOISE = 3,   /* in 0: UV; out 0: FLOAT */
    PMC_OP_MIX = 4,            /* in: FLOAT fac, COLOR a, COLOR b; out 0: COLOR */
    PMC_OP_MATH = 5,           /* in: FLOAT a, FLOAT b; out 0: FLOAT */
    PMC_OP_COLOR_RAMP = 6,     /* in 0: FLOAT fac; out 0: COLOR, out 1: FLOAT alpha */
    PMC_OP_NORMAL_MAP = 7,     /* in: COLOR, FLOAT strength; out 0: VECTOR (reads the hit normal) */
    PMC_OP_BSDF_OUTPUT = 8,    /* in: COLOR base colour, FLOAT roughness, VECTOR normal */
    PMC_OP_POSITION_NOISE = 9  /* no inputs (reads the hit's world position); out 0: FLOAT value
                                  noise of the position (freq, octaves, seed as the UV noises) */
};
enum pmc_math_op { PMC_MATH_ADD = 0, PMC_MATH_MUL = 1, PMC_MATH_POW = 2 };
#define PMC_NODE_CLAMP 1u      /* MATH: clamp the result to [0, 1] */

/* One input socket: a link to (node, socket) of the same material, or a constant. */
typedef struct pmc_input {
    int32_t node;              /* source node index in the material, or -1 = unconnected */
    uint32_t socket;           /* output socket of the source node */
    float value[3];            /* constant when unconnected (FLOAT uses value[0]);
                                  unconnected UV inputs read the hit UV and an
                                  unconnected VECTOR input reads the hit normal */
} pmc_input;                   /* 20 bytes */

typedef struct pmc_node_desc {
    uint32_t op;               /* enum pmc_op */
    uint32_t variant;          /* MATH: enum pmc_math_op; IMAGE_TEXTURE: texture index */
    uint32_t flags;            /* PMC_NODE_CLAMP */
    uint32_t seed;             /* noise seed */
    float freq;                /* noise base frequency f0 */
    uint32_t octaves;          /* noise octave count (1..8) */
    pmc_input in[3];
    float ramp_pos[8];         /* COLOR_RAMP stop positions, ascending */
    float ramp_rgba[8][4];     /* COLOR_RAMP stop colours */
} pmc_node_desc;               /* 244 bytes */

typedef struct pmc_texture_desc {
    const uint32_t* texels;    /* host, width*height RGBA8 texels (byte 0 = R), row 0 at v = 0 */
    uint32_t width, height;
} pmc_texture_desc;

typedef struct pmc_compile_opts {
    uint32_t min_subgraph_nodes;   /* smallest cacheable sub-graph (nodes besides UV inputs); 0 = 2 */
    uint32_t no_fold;              /* 1 = keep constant arithmetic nodes (no folding) */
    uint32_t texel_keys_only;      /* 1 = descriptors are UV texels only (Sec. 3.1): outputs that
                                      depend on the world position are not cached */
    uint32_t reserved[5];
} pmc_compile_opts;

#define PMC_MAX_CACHEABLE 8    /* cacheable outputs per material kept by the compiler */

typedef struct pmc_material_info {
    uint32_t n_nodes;          /* nodes given */
    uint32_t n_live;           /* nodes reachable from the sink */
    uint32_t n_folded;         /* constant nodes folded away (Sec. 2) */
    uint32_t n_instr;          /* interpreter instructions emitted */
    uint32_t n_regs;           /* per-lane float registers needed */
    uint32_t n_cacheable;      /* cacheable outputs K (Sec. 3) */
    uint32_t cacheable_node[PMC_MAX_CACHEABLE];
    uint32_t cacheable_socket[PMC_MAX_CACHEABLE];
    uint32_t subgraph_nodes[PMC_MAX_CACHEABLE];  /* sub-graph size of each, UV inputs excluded */
    uint32_t cacheable_type[PMC_MAX_CACHEABLE];  /* 0 FLOAT (raw float32 code), 1 COLOR (RGB9E5) */
    uint32_t cacheable_key[PMC_MAX_CACHEABLE];   /* 0 keyed by a UV texel (Sec. 3.1), 1 by a
                                                    world-space cell (the output depends on
                                                    the world position and not on UV) */
} pmc_material_info;

/* Create a context on HIP device `device`, or a host-only context when
 * device == -1 (compile and inspect graphs only; every device call then
 * returns PMC_ERR_STATE).  *out receives the context. */
pmc_status pmc_create(int device, pmc_ctx** out);
/* Destroy a context and everything it owns.  NULL is accepted.  While frame
 * graphs of the context exist, the context is only marked and is released with
 * the last of them. */
void pmc_destroy(pmc_ctx* ctx);
/* Message of the last failing call on ctx ("" if none).  Owned by ctx. */
const char* pmc_last_error(const pmc_ctx* ctx);
/* ABI version (PMC_ABI_VERSION) and sizeof of the public structs, by index
 * 0..20 (node_desc, input, texture_desc, compile_opts, material_info,
 * cache_params, shade_params, stats, hits, bsdf_out, debug_out, key_record,
 * frame_plan, tune_result, profile, surrogate_opts, surrogate_slot,
 * log_record, train_params, surrogate_stat, cone_hits); 0 for an unknown
 * index. */
uint32_t pmc_abi_version(void);
size_t pmc_abi_sizeof(uint32_t which);

/* Upload textures (copied into library-owned device memory; synchronous).
 * Replaces any previous set.  Graphs refer to textures by index.
 * PMC_ERR_STATE while frame graphs of the context exist. */
pmc_status pmc_set_textures(pmc_ctx* ctx, const pmc_texture_desc* tex, uint32_t n_tex);

/* Compile a graph set (Sec. 2 stack-machine form; Sec. 3 cacheable marking).
 * nodes: host array of all materials' nodes, material m owning
 * nodes[node_offsets[m] .. node_offsets[m+1]); node indices inside a
 * material are local.  Validates types, links and acyclicity
 * (PMC_ERR_GRAPH, message names material and node), folds constant MATH /
 * MIX / COLOR_RAMP nodes, marks cacheable outputs, computes the need masks
 * and registers and, on a device context, uploads the program
 * (synchronous).  Replaces any previous graph set.  opts may be NULL.
 * PMC_ERR_STATE while frame graphs of the context exist (they replay the
 * current program). */
pmc_status pmc_compile_materials(pmc_ctx* ctx, const pmc_node_desc* nodes,
                                 const uint32_t* node_offsets, uint32_t n_mats,
                                 const pmc_compile_opts* opts);
/* Compile report of one material (host). */
pmc_status pmc_get_material_info(const pmc_ctx* ctx, uint32_t mat, pmc_material_info* out);

/* ------------------------------------------------------------------ cache */

enum pmc_policy {
    PMC_POLICY_FIRST = 0,      /* keep the first inserted value (Sec. 3.2) */
    PMC_POLICY_OVERWRITE = 1,  /* evict the oldest-stamped entry of a full cell (16-byte entries) */
    PMC_POLICY_PRIORITY = 2    /* prefer samples of small path depth (Sec. 5 future work: keep
                                  directly visible samples when storage is short).  16-byte
                                  entries; the reserved word of an entry holds the depth
                                  (pmc_hits.bounce) of the sample that wrote it.  A full cell
                                  gives up its entry of the largest depth, then the oldest
                                  stamp, lowest index on ties; it is replaced when its depth
                                  is larger than the new sample's, or equal and written
                                  before the current frame */
};

typedef struct pmc_cache_params {
    uint64_t n_cells;          /* N_c >= 1 */
    uint32_t n_entries;        /* N_e in 1..64 */
    uint32_t entry_bytes;      /* 8: {u64 word}; 16: {u64 word, u32 stamp, u32 reserved=0} */
    uint32_t policy;           /* enum pmc_policy */
    int32_t level_bias;        /* integer offset added to floor(lambda) (Sec. 4 level offset) */
    uint32_t level_max;        /* levels clamp to [0, level_max]; 0 = 20 */
    uint32_t hash2_mask;       /* bits of the verification hash (Sec. 3.2) kept before the
                                  0 -> 1 step; 0 = all 32 bits (the method).  Fewer bits force
                                  the verification collisions that Sec. 3.2 says cannot be
                                  avoided, for tests of false hits */
} pmc_cache_params;

/* Create a table of n_cells * n_entries * entry_bytes bytes (16-byte entries
 * for OVERWRITE and PRIORITY: PMC_ERR_INVALID otherwise).  device_mem NULL:
 * the library allocates it; else the caller's device buffer of at least that
 * size (256-byte aligned) is used and stays caller-owned.  The table starts
 * cleared (synchronous).  Word layout: hash2 << 32 | 32-bit encoded value;
 * 0 = empty (Sec. 3.3). */
pmc_status pmc_cache_create(pmc_ctx* ctx, const pmc_cache_params* params, void* device_mem,
                            pmc_cache** out);
/* Destroy the handle (and the table if library-allocated).  NULL accepted.
 * Destroy every cache of a context before the context itself.  While frame
 * graphs replay into the table, it is only marked and is released with the
 * last of them. */
void pmc_cache_destroy(pmc_cache* cache);
/* Empty every entry (asynchronous on stream; a fill kernel, no memset node). */
pmc_status pmc_cache_clear(pmc_cache* cache, void* stream);
/* Device address and byte size of the table. */
pmc_status pmc_cache_device_ptr(pmc_cache* cache, void** ptr, size_t* bytes);
/* Copy the raw table to / from host memory (bytes must equal the table size);
 * both wait for the stream to finish the copy before returning. */
pmc_status pmc_cache_export(pmc_cache* cache, void* host_dst, size_t bytes, void* stream);
pmc_status pmc_cache_import(pmc_cache* cache, const void* host_src, size_t bytes, void* stream);

/* --------------------------------------------------------------- shading */

typedef struct pmc_hits {      /* all device pointers, caller-owned, n entries each */
    const uint32_t* material;  /* material id */
    const float* uv;           /* [n][2] */
    const float* duv;          /* [n][4]: g1.x, g1.y, g2.x, g2.y (ray-cone UV gradients, Sec. 3.1) */
    const float* normal;       /* [n][3] unit shading normal */
    uint64_t n;                /* hits; < 2^27 per call */
    const uint32_t* bounce;    /* [n] path depth of the hit (0 = seen from the camera), read
                                  only under PMC_POLICY_PRIORITY; NULL = all 0 */
    const float* position;     /* [n][3] world position; required (else PMC_ERR_INVALID) when
                                  the compiled graphs read it (POSITION_NOISE); NULL otherwise */
    const float* width;        /* [n] world-space footprint width (e.g. the ray cone's width at
                                  the hit); required with position.  A cacheable output that
                                  depends on the position is keyed by a world-space cell:
                                  level L from Eq. 1 with min(|g1|, |g2|) replaced by width,
                                  2^L cells per world unit, k0 with bit 7 set, k1 = (qx << 42 |
                                  qy << 21 | qz), each index mod 2^21 */
} pmc_hits;

typedef struct pmc_bsdf_out {  /* device pointers, caller-owned */
    float* base_color;         /* [n][3] */
    float* roughness;          /* [n] */
    float* normal;             /* [n][3] */
} pmc_bsdf_out;

/* Optional per-(hit, ordinal) diagnostics, device pointers (may be NULL). */
typedef struct pmc_debug_out {
    uint8_t* state;            /* [n][8]: 0 miss, 1 cache hit, 2 bypass, 3 no such ordinal,
                                  4 value from the surrogate network */
    float* value;              /* [n][8][3]: decoded value on a cache hit (unspecified otherwise) */
} pmc_debug_out;

enum pmc_mode {
    PMC_MODE_UNCACHED = 0,     /* plain evaluation; the table is not touched */
    PMC_MODE_CACHED = 1,       /* lookups and lock-free inserts race freely (Sec. 3.3) */
    PMC_MODE_SNAPSHOT = 2      /* lookups see the table as it was before the call; inserts
                                  are applied afterwards in (hit, ordinal) order: deterministic */
};
enum pmc_flags {
    PMC_FLAG_SORT = 1u,        /* sort hits by material first so each wave runs one program */
    PMC_FLAG_PERSISTENT = 2u,  /* a fixed grid of waves walks the work with a static stride */
    PMC_FLAG_DEFER = 4u,       /* cached modes: stage sparse misses per wave and evaluate them
                                  in dense passes (see defer_max) instead of in place */
    PMC_FLAG_LOG = 8u,         /* cached modes: append a pmc_log_record for each value of a
                                  surrogated output that is inserted (CACHED: the CAS or eviction
                                  succeeded; SNAPSHOT: a candidate was emitted) */
    PMC_FLAG_SURROGATE = 16u,  /* cached modes: a missed surrogated output of a trusted material
                                  takes its value from the material's network (not inserted);
                                  see the surrogate section below */
    PMC_FLAG_SURROGATE_INSERT = 32u  /* with PMC_FLAG_SURROGATE: the network's value is also
                                  inserted (Algorithm 1, or a snapshot candidate), so later
                                  lookups find it; the table then holds approximations within
                                  the trust threshold besides exact graph values */
};

typedef struct pmc_shade_params {
    uint32_t mode;             /* enum pmc_mode */
    uint32_t flags;            /* enum pmc_flags */
    uint32_t frame;            /* progressive pass index (stamps = frame + 1) */
    uint32_t chunk_waves;      /* run length: consecutive 64-hit chunks taken by one wave;
                                  0 = 4 with PMC_FLAG_DEFER, 1 otherwise */
    uint32_t blocks_per_cu;    /* persistent: resident blocks per CU; 0 = library choice */
    uint32_t defer_max;        /* PMC_FLAG_DEFER: a 64-hit chunk with more than defer_max
                                  missing lanes is evaluated where it was probed; sparser misses
                                  are staged per wave (in LDS) and evaluated together in dense
                                  passes over the wave's run.  0 = library default (48) */
    uint32_t waves_per_block;  /* flat grid: waves per workgroup, 1, 2 or 4 (a workgroup keeps
                                  its slot on the CU until its last wave ends); 0 = library
                                  default (4) */
    uint32_t reserved[1];
} pmc_shade_params;

typedef struct pmc_stats {     /* 64-bit counters, accumulated (+=) by pmc_shade */
    uint64_t hits_shaded;      /* hits processed */
    uint64_t probes;           /* lookups issued (cacheable outputs not bypassed) */
    uint64_t cache_hits;       /* lookups that found their key */
    uint64_t bypasses;         /* cacheable outputs that skipped the cache (non-finite input) */
    uint64_t inserts;          /* successful inserts (CAS from 0, or snapshot writes) */
    uint64_t cas_failures;     /* CAS that lost a race (nondeterministic mode) */
    uint64_t present;          /* insert found its key already stored */
    uint64_t cell_full;        /* insert found no free entry and did not evict */
    uint64_t overwrites;       /* OVERWRITE evictions */
    uint64_t nonfinite;        /* values not inserted because not finite */
    uint64_t candidates;       /* snapshot insert candidates */
    uint64_t nodes_executed;   /* lane-instructions executed by the interpreter */
    uint64_t nodes_total;      /* lane-instructions of full (uncached) evaluation */
    uint64_t invalid_material; /* hits with a material id out of range */
    uint64_t texture_evals;    /* lane evaluations of image-texture nodes (4 texel loads each) */
    uint64_t deferred;         /* hits staged for a dense evaluation after their probes */
    uint64_t insert_attempts;  /* finite values offered to the table (CAS or candidate) */
    uint64_t texture_evals_deferred;    /* texture_evals done while evaluating deferred hits */
    uint64_t insert_attempts_deferred;  /* insert_attempts made for deferred hits */
    uint64_t probes_deferred;  /* lookups repeated when a staged hit is evaluated */
    uint64_t surrogate_used;   /* missed outputs whose value came from a surrogate network */
    uint64_t logged;           /* records appended to the insert log */
    uint64_t audited;          /* surrogate-eligible misses evaluated by the graph instead, to
                                  measure the network's live error */
    uint64_t reserved[9];
} pmc_stats;                   /* 256 bytes */

/* Shade one batch (one progressive pass).  cache NULL or mode UNCACHED:
 * plain evaluation.  stats: device pmc_stats to accumulate into (NULL ok).
 * dbg: NULL, or device diagnostics buffers.  Asynchronous on stream. */
pmc_status pmc_shade(pmc_ctx* ctx, pmc_cache* cache, const pmc_hits* hits,
                     const pmc_bsdf_out* out, const pmc_shade_params* params,
                     pmc_stats* stats, const pmc_debug_out* dbg, void* stream);

/* For callers that cannot allocate device memory (code under their own HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * pmc_shade with the batch workspace (sorted order, the sort's bucket counts,
 * batch counters, statistics slots) in a fixed device array of
 * PMC_STATIC_SCRATCH_BYTES that every device the library runs on holds from
 * its first context until the process ends.  Same arguments, kernels and
 * results as pmc_shade, for modes UNCACHED and CACHED with flags SORT,
 * PERSISTENT and DEFER.  PMC_ERR_UNSUPPORTED, before anything is enqueued,
 * for SNAPSHOT mode, LOG or SURROGATE flags, more than PMC_STATIC_MAX_HITS
 * hits, or a sorted batch whose order and bucket counts (n + 2 (materials + 1)
 * words) do not fit the array.  Calls no hipMalloc or hipFree (the
 * caller passes inputs, outputs, stats and the table) and records no phase
 * timing.  All calls on one device share the array and each one overwrites
 * it: calls that overlap on one device (several streams, threads or
 * contexts) race and give undefined results. */
#define PMC_STATIC_SCRATCH_BYTES (16u << 20)
#define PMC_STATIC_MAX_HITS (1u << 20)
pmc_status pmc_shade_static(pmc_ctx* ctx, pmc_cache* cache, const pmc_hits* hits,
                            const pmc_bsdf_out* out, const pmc_shade_params* params,
                            pmc_stats* stats, const pmc_debug_out* dbg, void* stream);

/* Per-(hit, ordinal) descriptor fields, for bit-exact checks (Sec. 3.1, Eq. 1,
 * Sec. 3.2).  out: device array of n * 8 records; ordinals beyond the hit's
 * material K get bypass = 2.  Asynchronous. */
typedef struct pmc_key_record {
    uint32_t cell;             /* Hash(desc) % N_c */
    uint32_t hash2;            /* Hash2(desc), never 0 */
    int32_t level;             /* virtual mip level after bias and clamp */
    int32_t tx, ty;            /* virtual texel indices */
    uint32_t bypass;           /* 0 keyed, 1 bypassed (non-finite / out of range), 2 no ordinal */
} pmc_key_record;
pmc_status pmc_debug_keys(pmc_ctx* ctx, pmc_cache* cache, const pmc_hits* hits,
                          pmc_key_record* out, void* stream);

/* Algorithm 1 on raw descriptors: for i < n, insert (k0[i], k1[i]) -> the
 * 32-bit code enc[i] with one 64-bit compare-and-swap, all n concurrently.
 * desc = the two 64-bit descriptor words.  Device arrays.  Asynchronous. */
pmc_status pmc_cache_insert_raw(pmc_cache* cache, const uint64_t* k0, const uint64_t* k1,
                                const uint32_t* enc, uint64_t n, uint32_t frame,
                                pmc_stats* stats, void* stream);
/* Lookup of raw descriptors: hit[i] = 1 and enc_out[i] = code when found. */
pmc_status pmc_cache_lookup_raw(pmc_cache* cache, const uint64_t* k0, const uint64_t* k1,
                                uint64_t n, uint32_t* enc_out, uint8_t* hit, void* stream);

/* ------------------------------------------------------- progressive frames */

/* A progressive render: n_frames batches of hits_per_frame hits each, shaded
 * in order against one table (Sec. 1 and 3: values are inserted while frames
 * are rendered and reused by later frames). */
typedef struct pmc_frame_plan {
    pmc_hits hits;             /* device arrays of n_frames * hits_per_frame hits, frame-major
                                  (hits.n is ignored) */
    uint64_t hits_per_frame;   /* < 2^27 */
    uint32_t n_frames;
    uint32_t first_frame;      /* frame index of the first batch (stamps = frame + 1) */
    pmc_bsdf_out out;          /* device outputs */
    uint32_t out_per_frame;    /* 1: frame f writes entries [f * hits_per_frame, ...);
                                  0: every frame writes entries [0, hits_per_frame) */
    uint32_t clear_cache;      /* 1: empty the table before the first frame */
    pmc_shade_params params;   /* for every frame before late_frame; params.frame is ignored */
    pmc_stats* stats;          /* device counters accumulated by every frame, or NULL */
    uint32_t late_frame;       /* 0: params for every frame; else frames late_frame, ...
                                  (< n_frames) use late_params: once the table holds most
                                  values, other launch settings can be faster.  Same mode. */
    uint32_t reserved;
    pmc_shade_params late_params;
} pmc_frame_plan;

typedef struct pmc_frame_graph pmc_frame_graph;   /* opaque */

/* Capture the whole plan (table clear, then per frame: material sort, shade,
 * snapshot apply, statistics) into one HIP graph.  All device workspace is
 * reserved before capture; launches allocate nothing.  The plan's pointers are
 * baked into the graph and must stay valid while it is used.  Synchronous.
 * Until the graph is destroyed, the context keeps what it bakes in: compiling,
 * setting textures and surrogate setup return PMC_ERR_STATE, and so does a
 * shading call that would have to replace a workspace buffer (a larger batch
 * than any reserved so far); destroying the context or the table is deferred
 * to the graph's destruction. */
pmc_status pmc_frame_graph_create(pmc_ctx* ctx, pmc_cache* cache, const pmc_frame_plan* plan,
                                  pmc_frame_graph** out);
/* Replay the captured frames on `stream` (asynchronous). */
pmc_status pmc_frame_graph_launch(pmc_frame_graph* graph, void* stream);
/* Release the graph (waits for the device to finish its replays).  NULL
 * accepted. */
void pmc_frame_graph_destroy(pmc_frame_graph* graph);

/* Launch-parameter search.  Shades the plan's frames (without capture) under
 * each candidate setting of flags (persistence, deferral), chunk_waves,
 * defer_max and blocks_per_cu, timing each with HIP events (best of two
 * runs, the table cleared before each), and writes the fastest setting to
 * *best (mode taken from plan->params).  With plan->late_frame set, the
 * candidates replace late_params only (frames before late_frame keep
 * plan->params), which tunes the late frames on a table the early ones
 * filled.  The table is left cleared.  If json_path is not NULL, every
 * candidate and its time are written there as JSON.  Synchronous. */
typedef struct pmc_tune_result {
    pmc_shade_params best;     /* fastest setting found */
    double best_ms;            /* its time for the plan's frames */
    double default_ms;         /* time with the library defaults (flags = SORT) */
    uint32_t n_tried;
    uint32_t reserved;
} pmc_tune_result;
pmc_status pmc_autotune(pmc_ctx* ctx, pmc_cache* cache, const pmc_frame_plan* plan,
                        pmc_tune_result* out, const char* json_path);

/* ------------------------------------------------------ learned surrogate */

/* Beyond the paper, which caches exact sub-graph values only (Sec. 3): a small
 * per-material network may stand in for the deepest cacheable sub-graphs on a
 * cache miss.  The graph stays both the fallback and the judge of the
 * network's error.
 *
 *   surrogated outputs  cacheable outputs whose sub-graph has more than
 *                       min_subgraph_nodes nodes, packed in ordinal order into
 *                       4 channels (COLOR 3, FLOAT 1) while they fit; one
 *                       network ("slot") per material that has any
 *   features            x[4k..4k+3] = sin(w_k u), cos(w_k u), sin(w_k v), cos(w_k v),
 *                       w_k = 2 pi 2^(k-4), k = 0..7 (periods 16 .. 1/8 of a UV unit)
 *   network             h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3
 *                       with W1 64x32, W2 64x64, W3 4x64: 6532 parameters, stored
 *                       flat as W1 (row-major [out][in]), b1, W2, b2, W3, b3
 *   arithmetic          x, weights and activations in binary16 (round to nearest
 *                       even), products accumulated in FP32 on the matrix cores;
 *                       biases and the master weights in FP32
 *   training            mean squared error over the used channels of each sample,
 *                       Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the master
 *                       weights; batch sample i of step t is record
 *                       mix64(seed ^ (t << 32 | i)) mod n_train (SplitMix64 finalizer)
 *   trust               after training, the maximum absolute error over the
 *                       held-out records (used channels) must be <= max_err.
 *                       While shading with PMC_FLAG_SURROGATE, a hit h of frame f
 *                       with mix64(((f << 32) | h) ^ 0xD6E8FEB86659FD93) >> 58 == 0
 *                       (1 in 64) is evaluated by the graph instead, and the error of
 *                       the network there is recorded; a slot whose live error
 *                       exceeds max_err loses its trust after that call. */
typedef struct pmc_surrogate_opts {
    uint32_t min_subgraph_nodes;   /* surrogate outputs with larger sub-graphs; 0 = 32 */
    uint32_t log_capacity;         /* insert-log records, multiple of 64; 0 = 2^20 */
    uint64_t seed;                 /* He-uniform initialisation of every slot */
    float max_err;                 /* trust threshold (max abs error); 0 = 1e-2 */
    uint32_t reserved[3];
} pmc_surrogate_opts;

/* Choose the surrogated outputs of the compiled materials, create one slot per
 * material that has any, initialise their weights, and allocate the insert
 * log (device contexts).  Replaces an earlier setup.  Host-only contexts get
 * the slot table only.  *n_slots receives the slot count.  Synchronous.
 * PMC_ERR_STATE while frame graphs of the context exist. */
pmc_status pmc_surrogate_setup(pmc_ctx* ctx, const pmc_surrogate_opts* opts, uint32_t* n_slots);

typedef struct pmc_surrogate_slot {
    uint32_t material;
    uint32_t ordinal_mask;         /* bit c: cacheable ordinal c is surrogated */
    uint32_t n_channels;           /* channels used, 1..4 */
    uint32_t channel[8];           /* first channel of each surrogated ordinal */
    uint32_t reserved;
} pmc_surrogate_slot;
pmc_status pmc_surrogate_get_slot(const pmc_ctx* ctx, uint32_t slot, pmc_surrogate_slot* out);

/* Insert-log record (32 bytes): the exact UV of the hit and the FP32 value
 * the graph produced there (COLOR: value[0..2]; FLOAT: value[0]; rest 0). */
typedef struct pmc_log_record {
    uint32_t material;
    uint32_t ordinal;
    float u, v;
    float value[4];
} pmc_log_record;
/* Empty the log (asynchronous). */
pmc_status pmc_log_clear(pmc_ctx* ctx, void* stream);
/* Copy up to max records to host memory; *n gets the number held.  The log is
 * split into 64 regions filled independently; records come region by region.
 * Synchronous. */
pmc_status pmc_log_read(pmc_ctx* ctx, pmc_log_record* host_out, uint64_t max, uint64_t* n,
                        void* stream);

/* Master weights of a slot (6532 FP32 in the flat order above), host memory.
 * Setting them also resets the slot's Adam state and step count and clears
 * its trust.  Synchronous. */
pmc_status pmc_surrogate_set_params(pmc_ctx* ctx, uint32_t slot, const float* host_params);
pmc_status pmc_surrogate_get_params(pmc_ctx* ctx, uint32_t slot, float* host_params);
/* Force (trusted != 0) or clear a slot's trust.  Asynchronous. */
pmc_status pmc_surrogate_set_trust(pmc_ctx* ctx, uint32_t slot, int trusted, void* stream);

typedef struct pmc_train_params {
    uint32_t steps;                /* Adam steps per slot; 0 = 2000 */
    uint32_t batch;                /* samples per step, multiple of 128; 0 = 4096 */
    float lr;                      /* 0 = 1e-3 */
    uint32_t holdout;              /* held-out records per slot (at most a quarter of them);
                                      0 = 4096 */
    uint32_t min_records;          /* slots with fewer log records are skipped; 0 = 1024 */
    float lr_end;                  /* > 0: the step size decays geometrically from lr to lr_end
                                      over the call's steps; 0 = constant lr */
    uint64_t seed;                 /* batch sampling */
    uint32_t workgroups;           /* workgroups per slot, each taking a share of every step's
                                      batch, their gradient sums added in a fixed order before
                                      the step (data parallel, one cooperative launch); at most
                                      64 and batch / 128; 0 = as many as can be resident at
                                      once (at most 16), 1 = one workgroup per slot */
    uint32_t reserved;
} pmc_train_params;
/* Train every slot on its records of the insert log, all slots at once
 * (`workgroups` workgroups each): the log is grouped by slot, the last `holdout` records of
 * each group are held out, `steps` Adam steps are taken on the rest, and the
 * held-out error decides the trust.  Asynchronous; read the outcome with
 * pmc_surrogate_report. */
pmc_status pmc_surrogate_train(pmc_ctx* ctx, const pmc_train_params* params, void* stream);

/* The same training on caller records (device, n of them, all of the slot's
 * material), without hold-out or trust change.  Asynchronous. */
pmc_status pmc_surrogate_train_records(pmc_ctx* ctx, uint32_t slot, const pmc_log_record* records,
                                       uint32_t n, const pmc_train_params* params, void* stream);
/* Loss and gradient of the slot's current weights over exactly the n caller
 * records (device): grads (device, 6532 FP32, flat order) = dL/dparams with
 * L = sum over used channels (y - target)^2 / (number of used channels);
 * loss (device, 1 FP32).  Asynchronous. */
pmc_status pmc_surrogate_grad(pmc_ctx* ctx, uint32_t slot, const pmc_log_record* records,
                              uint32_t n, float* grads, float* loss, void* stream);
/* Network outputs y (device [n][4]) at uv (device [n][2]).  Asynchronous. */
pmc_status pmc_surrogate_infer(pmc_ctx* ctx, uint32_t slot, const float* uv, uint32_t n,
                               float* y, void* stream);

typedef struct pmc_surrogate_stat {
    uint32_t material;
    uint32_t trusted;
    uint32_t n_train;              /* records trained on by the last pmc_surrogate_train */
    uint32_t n_heldout;
    float max_err;                 /* held-out maximum / mean absolute error (used channels) */
    float mean_err;
    float loss;                    /* training loss of the last step */
    float live_max_err;            /* largest error seen on audited hits since the last training */
    uint32_t steps;                /* Adam steps taken since the weights were set */
    uint32_t live_checked;         /* audited outputs since the last training */
    uint32_t reserved[2];
} pmc_surrogate_stat;              /* 48 bytes */
/* Copy the per-slot statistics of slots [0, n) to host memory.  Synchronous. */
pmc_status pmc_surrogate_report(pmc_ctx* ctx, pmc_surrogate_stat* host_out, uint32_t n,
                                void* stream);

/* ------------------------------------------------------------ ray cones */

/* Texture-coordinate gradients of hits from their ray cones, for renderers
 * that track a cone per path (Sec. 3.1: the cone's intersection with the
 * surface is an ellipse; its two axes carried into UV space are g1 and g2,
 * after Akenine-Moller et al. 2021).  The surface is the hit triangle's plane
 * (normal e1 x e2); the ellipse of a cone of radius r around the ray has
 * semi-axes r / |cos| along the ray's projection onto the plane and r across
 * it, |cos| = |d.n| / (|d| |n|) clamped below at 1/1024; a ray within 1e-4 rad
 * of the normal uses the tangent frame of Duff et al. 2017 for the axes.  An
 * in-plane offset a moves the UV by du t1 + dv t2 with
 * du = ((a x e2).n) / (n.n), dv = ((e1 x a).n) / (n.n).  The output has the
 * layout of pmc_hits.duv (g1.x, g1.y, g2.x, g2.y), so it can be passed to
 * pmc_shade as is.  A degenerate triangle, a zero direction or a non-finite
 * input gives NaN gradients, which make the hit bypass the cache. */
typedef struct pmc_cone_hits {  /* device pointers, caller-owned, n entries each */
    const float* dir;          /* [n][3] ray direction (any length) */
    const float* radius;       /* [n] cone radius at the hit */
    const float* edge;         /* [n][6] triangle edges P1 - P0, then P2 - P0; 8-byte aligned */
    const float* uv_edge;      /* [n][4] UV edges uv1 - uv0, then uv2 - uv0; 16-byte aligned */
    uint64_t n;
} pmc_cone_hits;
/* duv: device [n][4], 16-byte aligned.  Asynchronous on stream. */
pmc_status pmc_ray_cone_gradients(pmc_ctx* ctx, const pmc_cone_hits* hits, float* duv,
                                  void* stream);

/* ------------------------------------------------------------- profiling */

/* Phase timing with HIP events recorded on the stream of each pmc_shade call,
 * around the launches of each phase.  Phases: 0 material sort, 1 shade
 * kernel, 2 snapshot apply, 3 statistics reduction. */
#define PMC_PROFILE_PHASES 4
typedef struct pmc_profile {
    double ms[PMC_PROFILE_PHASES];          /* accumulated milliseconds per phase */
    uint64_t launches[PMC_PROFILE_PHASES];  /* calls that recorded the phase */
} pmc_profile;
/* Start (on != 0) or stop recording.  Starting discards earlier records. */
pmc_status pmc_profile_enable(pmc_ctx* ctx, int on);
/* Wait for every recorded event, sum the phase times into *out, and, when
 * reset != 0, discard the records. */
pmc_status pmc_profile_read(pmc_ctx* ctx, pmc_profile* out, int reset);

#ifdef __cplusplus
}
#endif
#endif /* PMC_H */
