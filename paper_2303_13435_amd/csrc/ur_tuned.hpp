// Compile-time choices of the transform passes.  Written by
// paper_2303_13435_amd/tune.py from its timings on the GPU; the defaults
// below hold until a tuning run replaces them.
#pragma once

// pass X (binning, store and adjoint column passes): threads' worth of
// columns per block for columns of one wavefront (1024 points)
#ifndef UR_X_THREADS
#define UR_X_THREADS 256
#endif

// pass X with binning: minimum resident waves per SIMD (a VGPR cap; 1 = none)
// threads per block of the binning x pass for 2048-point columns (two
// wavefronts per column)
#ifndef UR_X_THREADS_2K
#define UR_X_THREADS_2K 256
#endif

// forward y pass of 2048-point columns: half-width tiles (1) or full
#ifndef UR_Y_HALF_2K
#define UR_Y_HALF_2K 0
#endif

#ifndef UR_X_MINW_F32
#define UR_X_MINW_F32 3
#endif
#ifndef UR_X_MINW_F64
#define UR_X_MINW_F64 1
#endif

// pass Z, real FP32 columns up to 1024 points: pencil pairs per block (a
// tile of twice as many y rows)
#ifndef UR_Z_PAIRS_F32
#define UR_Z_PAIRS_F32 4
#endif

// pass Z: deal the two tiles that share a 128-byte line of A (tiles of
// fewer than 16 FP32 rows) to blocks that run on the same XCD
#ifndef UR_Z_XCD
#define UR_Z_XCD 0
#endif

// the inverse z passes of the adjoint (inverse transform, fold onto the
// cell): pencil pairs per block of real FP32 columns up to 1024 points
#ifndef UR_ZI_PAIRS_F32
#define UR_ZI_PAIRS_F32 8
#endif

// streaming (non-temporal) policy: stores of the first intermediate (pass
// Z), stores of the second (pass Y), column loads of passes Y and X
#ifndef UR_ST_NT_A
#define UR_ST_NT_A 1
#endif
#ifndef UR_ST_NT_B
#define UR_ST_NT_B 1
#endif
// zero-extended column loads of the y passes and of the x passes: 1 skips
// chunks wholly outside the valid range with a scalar branch, 0 loads every
// chunk from a resource that starts at the first valid element
#ifndef UR_LD_SKIP_Y
#define UR_LD_SKIP_Y 1
#endif
#ifndef UR_LD_SKIP_X
#define UR_LD_SKIP_X 0
#endif

#ifndef UR_LD_NT
#define UR_LD_NT 1
#endif

// pass X: twiddles and LDS offsets reloaded per column (1) or held in
// registers across the column loop (0)
#ifndef UR_X_REFETCH
#define UR_X_REFETCH 0
#endif

// adjoint x pass: twiddles and LDS offsets reloaded per column (1) or held in
// registers across the column loop (0)
#ifndef UR_XADJ_REFETCH
#define UR_XADJ_REFETCH 0
#endif
