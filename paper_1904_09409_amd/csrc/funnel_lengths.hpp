// funnel_lengths.hpp -- transform lengths with compiled kernels, in groups
// that are built as separate translation units.  Every length is 7-smooth.
#pragma once

#define FUNNEL_LENGTHS_G0(X) X(8) X(16) X(24) X(32) X(40) X(48) X(64) X(80) X(96) X(128) X(160) X(192)
#define FUNNEL_LENGTHS_G1(X) X(240) X(256) X(320) X(384) X(480) X(512) X(560)
#define FUNNEL_LENGTHS_G2(X) X(640) X(720) X(768) X(1024) X(1080)
#define FUNNEL_LENGTHS_G3(X) X(1120) X(1280) X(1536) X(1920)
#define FUNNEL_LENGTHS_G4(X) X(2000) X(2048)
#define FUNNEL_LENGTHS_G5(X) X(3000) X(4096)

#define FUNNEL_LENGTHS(X) \
  FUNNEL_LENGTHS_G0(X) FUNNEL_LENGTHS_G1(X) FUNNEL_LENGTHS_G2(X) FUNNEL_LENGTHS_G3(X) FUNNEL_LENGTHS_G4(X) \
      FUNNEL_LENGTHS_G5(X)
