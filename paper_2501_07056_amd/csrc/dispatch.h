// Type dispatch over the index and value types of A and B.
#pragma once

#define MG_DISPATCH3(M, ...)                                                 \
  do {                                                                        \
    if (!(M).rp64 && !(M).col64) {                                            \
      using RP = int32_t; using CI = int32_t;                                 \
      if ((M).f64) { using V = double; __VA_ARGS__; } else { using V = float; __VA_ARGS__; } \
    } else if (!(M).rp64 && (M).col64) {                                      \
      using RP = int32_t; using CI = int64_t;                                 \
      if ((M).f64) { using V = double; __VA_ARGS__; } else { using V = float; __VA_ARGS__; } \
    } else if ((M).rp64 && !(M).col64) {                                      \
      using RP = int64_t; using CI = int32_t;                                 \
      if ((M).f64) { using V = double; __VA_ARGS__; } else { using V = float; __VA_ARGS__; } \
    } else {                                                                  \
      using RP = int64_t; using CI = int64_t;                                 \
      if ((M).f64) { using V = double; __VA_ARGS__; } else { using V = float; __VA_ARGS__; } \
    }                                                                         \
  } while (0)

#define MG_DISPATCH2(M, ...)                         \
  do {                                                \
    if (!(M).rp64 && !(M).col64) {                    \
      using RP = int32_t; using CI = int32_t; __VA_ARGS__;   \
    } else if (!(M).rp64 && (M).col64) {              \
      using RP = int32_t; using CI = int64_t; __VA_ARGS__;   \
    } else if ((M).rp64 && !(M).col64) {              \
      using RP = int64_t; using CI = int32_t; __VA_ARGS__;   \
    } else {                                          \
      using RP = int64_t; using CI = int64_t; __VA_ARGS__;   \
    }                                                 \
  } while (0)

