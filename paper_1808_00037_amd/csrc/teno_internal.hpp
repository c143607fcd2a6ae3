// teno_internal.hpp -- host-side context layout shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include "teno.h"
#include "teno_device.hpp"

#include <utility>
#include <vector>

struct teno_ctx {
    teno_grid grid;
    teno_opts opts;
    hipStream_t stream = nullptr;
    int nv = 1;
    int num_cu = 256;
    double dx = 1, dy = 1, eps_x = 0, eps_y = 0;
    size_t ncell = 0, nelem = 0, nfx = 0, nfy = 0, esize = 8;
    teno::Ctrl *ctrl_d = nullptr;
    void *S1 = nullptr, *S2 = nullptr, *dUy = nullptr;
    // adjoint scratch (stage states of one checkpoint segment, adjoint work arrays)
    void *adj_scratch = nullptr;
    size_t adj_scratch_bytes = 0;
    // captured step graph
    hipStream_t cap_stream = nullptr;   // private stream used only to capture graphs
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    void *graph_U = nullptr;
    double graph_dt = 0.0;
    // kernel timing (eager launches only)
    bool timing = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> events;
    size_t events_used = 0;
};

// One sweep launch request (see teno_lib.hip).
struct SweepReq {
    int dir;
    int mode;
    int stage;
    bool frozen;
    const void *U, *U0, *addend;
    void *out, *Fout, *chi_out;
    uint32_t *masks_out, *flags_out;
    const uint32_t *masks_in;
    const double *alpha;
    unsigned long long *part;
};

bool teno_validate(const teno_grid *g, const teno_opts *o);
bool teno_validate_opts(const teno_opts *o);
// The Lax-Friedrichs constants' form: one constant max(|u_n| + c) for every field when asked for,
// and always for the reconstruction per conserved component (every component needs the fastest wave).
inline int teno_alpha_mode(const teno_opts &o) { return (o.alpha_mode || !o.characteristic) ? 1 : 0; }
void teno_fill_derived(teno_ctx *c);
teno_status teno_ensure_scratch(teno_ctx *c);
void teno_launch_sweep(teno_ctx *c, const SweepReq &r);
void teno_launch_wavespeed(teno_ctx *c, const void *U, int ring);
void teno_launch_prep(teno_ctx *c, int ring, int stage, double dt_fixed, const double *frozen, double *record);
void teno_launch_clear(teno_ctx *c, int ring);
void teno_enqueue_step(teno_ctx *c, void *U, double dt_fixed, const double *frozen_ad, double *record_ad,
                       uint32_t *masks_rec, const uint32_t *masks_in, void **stage_states);
