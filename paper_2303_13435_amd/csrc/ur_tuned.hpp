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
#ifndef UR_X_MINW_F32
#define UR_X_MINW_F32 3
#endif
#ifndef UR_X_MINW_F64
#define UR_X_MINW_F64 2
#endif

// pass Z, real FP32 columns up to 1024 points: pencil pairs per block (a
// tile of twice as many y rows)
#ifndef UR_Z_PAIRS_F32
#define UR_Z_PAIRS_F32 4
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
#ifndef UR_LD_NT
#define UR_LD_NT 1
#endif
