// dco_batch.h -- data shared by the batched matcher's host code (batch.cpp)
// and its persistent kernel (k_batch.hip).
#pragma once

#include "dco_internal.h"

constexpr int kBatchStages = 5;  // census, records, cost + aggregation, WTA, LR
constexpr int kWtaPx = 4096;     // pixels per WTA item
constexpr int kLrRows = 2;       // rows per LR item
constexpr int kXcds = 8;         // accelerator dies; workgroup b runs on XCD b % 8

// Static description and scratch of one pair.
struct BatchPair {
    int W, H, D, nstrips;
    int band;     // output rows per aggregation item (tuned)
    int dchunk;   // disparities per aggregation item (tuned)
    int nitems[kBatchStages];
    uint32_t* arms[2];
    uint4* pix[2];   // packed pixels: census lo, census hi, RGB, 8 L_min
    AggRecords rec[2];
    float* agg[2];
    int16_t* dint[2];
    float* delta;
};

// Inputs and outputs of one pair for the current call.
struct BatchIO {
    const uint8_t* L;
    const uint8_t* R;
    float* disp;
    uint8_t* valid;
};

struct BatchItem {
    int pair, stage, view, a, b, c;
};

struct BatchArgs {
    const BatchPair* pairs;
    const BatchIO* io;
    const BatchItem* items;   // stage-ordered work list
    const float* tabA;
    const float* tabC;
    const float* alpha;
    const float* beta;
    int cw, ch, L1, tau1, subpixel, maxdiff;
    // stage 2: XCD x runs items [xsplit[x], xsplit[x + 1]) (absolute indices);
    // the parts are contiguous runs of one (pair, view, strip, band) with
    // neighbouring disparities, of about equal cost
    int xsplit[kXcds + 1];
};

// Launches the five stage kernels on `st`: stage s handles items
// [first[s], first[s + 1]) with grid[s] workgroups (stage 2: one per item,
// kXcds times the largest per-XCD part).
hipError_t launch_batch(const BatchArgs& a, int iters, const int* first, const int* grid,
                        hipStream_t st);
// Resident workgroups per CU of each stage kernel.
void batch_blocks_per_cu(int iters, int* per_stage);
