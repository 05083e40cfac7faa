// The whole library is one translation unit, so device globals (the error
// word, the empty brick) need no relocatable device code.
#include "api.hip"
#include "voxelize.hip"
#include "jfa.hip"
#include "select.hip"
#include "scene.hip"
#include "instance.hip"
#include "trace.hip"
#include "lbvh.hip"
#include "distance.hip"
#include "shadow.hip"
#include "batch.hip"
#include "graph.hip"
