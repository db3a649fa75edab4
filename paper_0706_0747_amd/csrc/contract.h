// Declarations shared by the contraction kernel (contract.hip) and the apply driver (apply.hip).
// Internal to libmwns.
#pragma once
#include "mwns_internal.h"

namespace mwns {

typedef unsigned int u4 __attribute__((ext_vector_type(4)));

// One contraction job of a level: a box of coarse displacements, a fine-displacement mask, a
// term range and the band it belongs to.
struct Tpl {
    int lo[3], hi[3];      // coarse displacement box
    int mlo[3], mhi[3];    // fine displacement mask per dimension
    int m1, m2;            // inclusive term range
    int dpart;             // 0: whole band (all children, +), 1: down band (internal children, -)
    int prec;              // precision class of the job's terms (PREC_*)
};

// Entry d of a per-dimension triple of a job (the same in every lane), without indexing the array at
// run time: a private array indexed with a run-time value is placed in scratch memory, and the
// compiler turns a select between the entries back into such an index unless each entry is first
// read into a register on its own.
__device__ inline int pick3(const int (&a)[3], int d) {
    const int a0 = __builtin_amdgcn_readfirstlane(a[0]), a1 = __builtin_amdgcn_readfirstlane(a[1]);
    const int a2 = __builtin_amdgcn_readfirstlane(a[2]);
    return d == 0 ? a0 : (d == 1 ? a1 : a2);
}

// Precision classes of a job.  Every class accumulates into the FP64 output; the reduced ones
// take their inputs from FP32 or split-BF16 copies of the input bricks and accumulate each
// mode product in FP32.
enum { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16C = 2, PREC_BF16 = 3, NPREC = 4 };

constexpr int NMAX = 4;            // largest box extent per dimension of one job (the driver splits boxes)

// One level of one apply as seen by the contraction kernel.
struct LevelDesc {
    const double* Xr;        // real input bricks of the level (the level's own bricks)
    const double* Xg;        // ghost input bricks
    const float* Xr32;       // FP32 copies (or null): rows padded to 16, [brick][v1][v2][16] (k <= KNARROW)
    const float* Xg32;
    const u4* Xrb;           // split-BF16 copies: [brick][v1][v2][4 groups] of (4 hi, 4 lo)  (or null)
    const u4* Xgb;
    const int32_t* nbr;      // [brick][(2Lr+1)^3] input index, -1 outside the cube
    const uint8_t* cmask;    // [brick] bit s set when child s is internal
    const Tpl* tpl;          // jobs of the level
    const double* Fj;        // F^{j;m,l} of the level [M][NLF][k][k]
    const double* w;         // weights w_m of the operator
    double* out;             // output bricks of the level
    int64_t nreal;
    int Lr, valid, ntpl, pad;
};

constexpr int NXCD = 8;            // XCDs of the MI355X; workgroup b is dispatched to XCD b % 8

// Work queues of the persistent launch: counters[8] | begin[8] | end[8] (ints).  Queue x holds
// the positions [begin[x], end[x]) of the order array; counters start at zero.
constexpr int QUEUE_INTS = 3 * NXCD;

template <template <int> class Fn, class... Args>
void dispatch_k(int k, Args&&... args) {
    switch (k) {
        case 1: Fn<1>::run(args...); break;
        case 2: Fn<2>::run(args...); break;
        case 3: Fn<3>::run(args...); break;
        case 4: Fn<4>::run(args...); break;
        case 5: Fn<5>::run(args...); break;
        case 6: Fn<6>::run(args...); break;
        case 7: Fn<7>::run(args...); break;
        case 8: Fn<8>::run(args...); break;
        case 9: Fn<9>::run(args...); break;
        case 10: Fn<10>::run(args...); break;
        default: fail(MWNS_EINVAL, "unsupported k");
    }
}

int num_variants();
int variant_for(const mwns_ctx* ctx, int k);

// The jobs of precision class prec of every listed (level, brick).  queues == nullptr: workgroup
// b takes order[b] (nblocks = number of listed bricks); otherwise nblocks resident workgroups pull
// positions from the 8 per-XCD queues (their own XCD's first, then the others') until all are
// drained.  accumulate: add to the output brick instead of overwriting it.  The tile variant
// applies to the FP64 class; the reduced classes run in the shape of variant 0 (8 waves, two
// workgroups per CU).
void launch_contract(int k, int variant, int prec, bool accumulate, hipStream_t st, int64_t nblocks,
                     const LevelDesc* levels, const int2* order, int* queues);
// Workgroups of that kernel that fit on the device at once (for the persistent launch).
int64_t resident_blocks(int k, int variant, int prec, int device);
// The whole-brick contraction kernel for KNARROW < k <= KMAX (2k = 18, 20: 16-wide tiles plus
// 4-row tails), classes PREC_F64 and PREC_F32 (which adds to the output): one workgroup per output
// brick, order[] entries (level descriptor, brick); variant 0 four waves loading the next input
// slice ahead, 1 eight waves in two groups on alternate terms, 2 as 0 loading each slice when it is
// needed.  queues as in launch_contract.
int num_wide_variants();
void launch_contract_wide(int k, int variant, int prec, hipStream_t st, int64_t nblocks, const LevelDesc* levels,
                          const int2* order, int* queues);
int64_t resident_blocks_wide(int k, int variant, int prec, int device);
// FP32 or split-BF16 copies of input bricks, 16-byte groups as the one-tile kernel reads them, for
// several arrays in one launch: entry i converts nb[i] bricks X[i] into out[i] (split BF16 when
// bf[i]); the launch gives entry i the 256-thread blocks [bstart[i], bstart[i + 1]).
constexpr int MAXCONV = 4 * (MAXLEV + 1);
struct ConvTab {
    int n = 0;
    int bf[MAXCONV];
    int64_t nb[MAXCONV];
    int64_t bstart[MAXCONV + 1];
    const double* X[MAXCONV];
    u4* out[MAXCONV];
    // appends nb bricks X -> out (nothing for nb = 0)
    void add(int k, int64_t nbricks, const double* x, u4* o, bool split) {
        if (nbricks <= 0) return;
        const int64_t blocks = (nbricks * 2 * k * 2 * k * 4 + 255) / 256;
        if (n == 0) bstart[0] = 0;
        bf[n] = split;
        nb[n] = nbricks;
        X[n] = x;
        out[n] = o;
        bstart[n + 1] = bstart[n] + blocks;
        ++n;
    }
};
void launch_convert(int k, hipStream_t st, const ConvTab& tb);

}  // namespace mwns
