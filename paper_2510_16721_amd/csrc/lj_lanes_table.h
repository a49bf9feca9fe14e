// LJ lanes per atom by band size (atoms x images at creation): the fastest lane
// count of an FP32 LJ band stepped alone.  Written by tune_lanes.py from
// force-stage times (us per step) of LJ FCC vacancy-hop bands:
//         217 atom-images: 1:     40.2  2:     23.7  4:     17.4  8:     14.5
//         749 atom-images: 1:     40.5  2:     24.4  4:     25.5  8:     26.4
//        1785 atom-images: 1:     39.7  2:     38.6  4:     40.7  8:     42.3
//        6041 atom-images: 1:     28.2  2:     28.2  4:     29.9  8:     32.8
//       14329 atom-images: 1:     29.4  2:     29.3  4:     31.6  8:     34.2
//       37261 atom-images: 1:     29.0  2:     28.4  4:     30.9  8:     33.4
//      114681 atom-images: 1:     37.9  2:     37.8  4:     41.5  8:     45.3
//      298137 atom-images: 1:     52.7  2:     69.9  4:     76.7  8:     83.2
//      682885 atom-images: 1:    104.2  2:    123.1  4:    136.4  8:    148.4
//     2341320 atom-images: 1:    449.6  2:    516.9  4:    563.1  8:    603.9
#ifndef CFNEB_LJ_LANES_TABLE_H
#define CFNEB_LJ_LANES_TABLE_H

struct LjLanesEntry {
    long long max_atom_images;
    int lanes;
};
static const LjLanesEntry kLjLanesTable[] = {
    {403LL, 8},
    {1156LL, 2},
    {9223372036854775807LL, 1},
};

#endif
